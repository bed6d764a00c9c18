"""Benchmark: the even-odd preconditioned Wilson normal operator on one MI355X.

A step is one application of Mhat^dagger Mhat, Mhat = 1 - kappa^2 D_eo D_oe, on
a 32^3 x 64 lattice with FP32 storage and 12-real links (eps = 0.5,
kappa = 0.124): four even-odd dslash launches (two fused with the
1 - kappa^2 update), the inner operator of the CG solver.  Flops follow the
1320-per-site dslash convention: 2 * (2 * 1320 + 48) per even site per step.

Prints one JSON line with the throughput, the roofline of the dslash kernel
(algorithmic HBM bytes per launch over its average duration, timed with HIP
events on the stream the kernels run on) and the FP64 CPU oracle timed on
the host on the same operator.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--shape-sweep-only] [--precision-sweep-only]
                    [--multi-rhs-only] [--network-only]
"""
import argparse
import json
import os
import platform
import sys
import time

DIMS = (32, 32, 32, 64)
EPS, KAPPA = 0.5, 0.124
BC = (1, 1, 1, -1)
FLOPS_DSLASH = 1320          # per output site
FLOPS_XPAY = 48              # a x + b y on 24 reals
# algorithmic HBM bytes per output site of one FP32 12-real EO dslash:
# 8 links x 48 B + input spinor 96 B (each read once) + output 96 B; xpay adds 96 B
BYTES_DSLASH = 8 * 48 + 96 + 96
BYTES_XPAY = 96
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--dims", type=int, nargs=4, default=list(DIMS))
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--no-extras", action="store_true", help="skip the multi-rhs and ragged-batch measurements")
    ap.add_argument("--no-sweep", action="store_true", help="skip the L^3 x 2L volume sweep")
    ap.add_argument("--precision-sweep-only", action="store_true",
                    help="only the EO dslash at every storage precision on the benchmark lattice (for counter runs)")
    ap.add_argument("--shape-sweep-only", action="store_true",
                    help="only the EO dslash over lattices one extent short of 32^3 x 64 (for counter runs)")
    ap.add_argument("--multi-rhs-only", action="store_true",
                    help="only the 16-rhs records on 16^3 x 32 (per-rhs and matrix-core paths; for counter runs)")
    ap.add_argument("--network-only", action="store_true",
                    help="only the learned preconditioner's network applied on 32^3 x 64 and 16^3 x 32 (for counter runs)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON tuning table: loaded if it exists (no tuning), else tuned and written there")
    return ap.parse_args()


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_0810_5365_amd", "csrc")
    # everything that shapes the timed launches: the kernel body, its launcher, device helpers,
    # the host core, the tuner that picks the launch shapes, and the step's composition
    for f in ("dslash_body.h", "dslash.hip", "wd_device.h", "wd_core.h", "tune.hip", "api.hip"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()


def measured_traffic(dims):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the kernel sources as they are now (else None)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "dslash_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256") != kernel_source_sha() or tuple(dims) != (32, 32, 32, 64):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(U, psi_e, dims, gpu_out=None):
    """The FP64 oracle's Mhat^dagger Mhat on the same inputs (one application), and the
    relative L2 distance of the benchmark step's FP32 output from it."""
    import oracle as orc
    Vh = psi_e.shape[0]
    orc.parity_sites(dims, 0)
    orc.parity_sites(dims, 1)   # build the checkerboard index tables outside the timing
    t0 = time.perf_counter()
    reps = 0
    while True:
        ref = orc.mhat_dag_mhat(U, psi_e, KAPPA, BC)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 3:
            break
    dt = (time.perf_counter() - t0) / reps
    flops = Vh * 2 * (2 * FLOPS_DSLASH + FLOPS_XPAY)
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": "%d application(s) of the FP64 oracle's Mhat^dag Mhat on the full %dx%dx%dx%d lattice "
                      "(%d even sites), %.2f s each" % (reps, *dims, Vh, dt),
            "one_core": cpu_one_core(),
            "eo_dslash_fp64_vs_fp32_build": cpu_eo_dslash(U, psi_e, dims),
            "step_rel_l2_vs_oracle": None if gpu_out is None else float(orc.rel_l2(gpu_out, ref))}


def cpu_eo_dslash(U, psi_e, dims, reps=3):
    """The oracle's even-output hopping term D_eo (odd input) on all host cores, from the FP64
    build and from the single-precision build of the same source (the CPU counterpart of the
    FP32 operator): median of `reps` calls each, GFLOP/s at 1320 flops per even site."""
    import numpy as np
    import oracle as orc
    Vh = psi_e.shape[0]
    full = orc.eo_merge(np.zeros_like(psi_e), psi_e, dims)   # the source on the odd sites
    U32, full32 = U.astype(np.complex64), full.astype(np.complex64)   # converted outside the timing
    res = {}
    for name, fn in (("fp64", lambda: orc.dhop(U, full, BC, out_parity=0)),
                     ("fp32_build", lambda: orc.dhop_fp32(U32, full32, BC, out_parity=0))):
        fn()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        dt = float(np.median(ts))
        res[name] = {"gflops": round(Vh * FLOPS_DSLASH / dt / 1e9, 3), "s_median": round(dt, 4)}
    res.update({"cores": orc.num_threads(), "lattice": list(dims),
                "sample": "%d calls of D_eo per build on %dx%dx%dx%d" % (reps, *dims)})
    return res


_ONE_CORE = r"""
import sys, time
sys.path.insert(0, sys.argv[1])
import lattice_synth as ls, oracle as orc
dims = (16, 16, 16, 32)
U = ls.gauge_field(dims, 0.5, ls.link_seed(2))
psi = ls.gaussian_complex((16 * 16 * 16 * 16, 4, 3), ls.source_seed(2), ls.STREAM_SPINOR)
orc.mhat_dag_mhat(U, psi, 0.124, (1, 1, 1, -1))
t0 = time.perf_counter()
orc.mhat_dag_mhat(U, psi, 0.124, (1, 1, 1, -1))
print(orc.num_threads(), time.perf_counter() - t0)
"""


def cpu_one_core():
    """The same oracle operator on one thread (a child process with OMP_NUM_THREADS=1),
    on 16^3 x 32 to keep it to a few seconds."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", HIP_VISIBLE_DEVICES="")
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        out = subprocess.run([sys.executable, "-c", _ONE_CORE, root], env=env, capture_output=True, text=True,
                             timeout=300, check=True).stdout.split()
    except (subprocess.SubprocessError, OSError) as e:
        return {"error": str(e)[:200]}
    threads, dt = int(out[0]), float(out[1])
    Vh = 16 * 16 * 16 * 16
    return {"value": round(Vh * 2 * (2 * FLOPS_DSLASH + FLOPS_XPAY) / dt / 1e9, 3), "unit": "GFLOP/s",
            "cores": threads, "sample": "1 application of Mhat^dag Mhat on 16x16x16x32, %.2f s" % dt}


def plaquette(U):
    """Average plaquette (1/3) Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag over
    sites and the six planes, periodic wrap (a property of the gauge field alone,
    reported beside each solve)."""
    import numpy as np
    axis = {0: 3, 1: 2, 2: 1, 3: 0}   # mu = x, y, z, t -> array axis of (T, Z, Y, X)
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = U[mu] @ np.roll(U[nu], -1, axis[mu])
            b = U[nu] @ np.roll(U[mu], -1, axis[nu])
            tot += float((a * b.conj()).real.sum())   # Re tr(a b^dag)
    return float(tot / (6 * 3 * U[0].shape[0] * U[0].shape[1] * U[0].shape[2] * U[0].shape[3]))


def timed_repeats(fn, stream, torch, n=100, repeats=5, warmup=10):
    """Median and minimum over `repeats` runs of n back-to-back calls (HIP events on
    the stream), microseconds per call."""
    import numpy as np
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    us = []
    for _ in range(repeats):
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        us.append(e0.elapsed_time(e1) * 1e3 / n)
    return float(np.median(us)), float(min(us))


# lattices one extent short of 32^3 x 64 (and 28^4 x 2): the rate against the extents
SHAPE_SWEEP = ((24, 32, 32, 64), (28, 32, 32, 64), (30, 32, 32, 64), (32, 24, 32, 64), (32, 28, 32, 64),
               (32, 32, 28, 64), (32, 32, 32, 56), (28, 28, 28, 56), (32, 32, 32, 64))


# algorithmic bytes per even output site of one 12-real EO dslash by storage precision
# (8 links + input + output; 16-bit: 12 reals x 2 B per link, 24 x 2 B + a 4 B scale per spinor)
BYTES_BY_PREC = {"f64": 8 * 96 + 192 + 192, "f32": BYTES_DSLASH, "f16": 8 * 24 + 52 + 52, "bf16": 8 * 24 + 52 + 52,
                 "f32_r18": 8 * 72 + 96 + 96, "f16_r18": 8 * 36 + 52 + 52, "bf16_r18": 8 * 36 + 52 + 52}


def dslash_by_precision(w, ctx, stream, torch, ls, g, dims, psi_o, U=None, tune=True):
    """The EO dslash D_eo (no dagger, no update) at every storage precision on the benchmark's
    field and source, autotuned: median and minimum of five runs of 100 launches, GFLOP/s at
    1320 flops per site, algorithmic GB/s and fraction of the HBM peak; with the links U also
    FP32 with 18-real links."""
    X, Y, Z, T = dims
    Vh = X * Y * Z * T // 2
    lat = w.lattice(dims, BC)
    rows = {}
    for prec in (w.F64, w.F32, w.F16, w.BF16):
        name = w.PREC_NAMES[prec]
        g.prepare(prec)
        fin = w.pack(ctx, lat, w.ODD, prec, psi_o)
        fout = w.new_field(lat, w.EVEN, prec)
        if tune:
            w.wd_autotune_dslash(g.handle, prec, 1, None)
        med, mn = timed_repeats(lambda: w.wd_dslash(g.handle, w.EVEN, 0, prec, 1, fin.data_ptr(), fout.data_ptr()),
                                stream, torch)
        b = BYTES_BY_PREC[name]
        rows[name] = {"us_median": round(med, 3), "us_min": round(mn, 3),
                      "gflops": round(Vh * FLOPS_DSLASH / med / 1e3, 1), "bytes_per_site": b,
                      "gbs_algorithmic": round(Vh * b / med / 1e3, 1),
                      "frac_hbm": round(Vh * b / med / 1e3 / HBM_PEAK_GBS, 4),
                      "tuned": w.tune_get(ctx, w.dslash_key(dims, prec, 12, 1, 0, 0))}
        del fin, fout
    if U is not None:
        # 18-real links: no row rebuild, 50% more link bytes
        g18 = w.Gauge(ctx, dims, BC, w.RECON_18)
        g18.upload(U)
        for prec in (w.F32, w.F16, w.BF16):
            name = w.PREC_NAMES[prec] + "_r18"
            g18.prepare(prec)
            fin = w.pack(ctx, lat, w.ODD, prec, psi_o)
            fout = w.new_field(lat, w.EVEN, prec)
            if tune:
                w.wd_autotune_dslash(g18.handle, prec, 1, None)
            med, mn = timed_repeats(lambda: w.wd_dslash(g18.handle, w.EVEN, 0, prec, 1, fin.data_ptr(), fout.data_ptr()),
                                    stream, torch)
            b = BYTES_BY_PREC[name]
            rows[name] = {"us_median": round(med, 3), "us_min": round(mn, 3),
                          "gflops": round(Vh * FLOPS_DSLASH / med / 1e3, 1), "bytes_per_site": b,
                          "gbs_algorithmic": round(Vh * b / med / 1e3, 1),
                          "frac_hbm": round(Vh * b / med / 1e3 / HBM_PEAK_GBS, 4),
                          "tuned": w.tune_get(ctx, w.dslash_key(dims, prec, 18, 1, 0, 0))}
            del fin, fout
        g18.close()
    return {"lattice": list(dims), "kernel": "dslash_kernel<P, r12> and <P, r18>, D_eo", **rows}


def single_launch_us(run, stream, torch, cold, n=20):
    """One launch at a time between events (median and minimum over n, microseconds):
    warm = right after another launch of the same call, so whatever of its working set the
    caches kept is still there; cold = after evicting it with a 1 GiB write and then a
    1 GiB read of other buffers (so that no dirty line of the write is still being written
    back when the launch starts)."""
    import numpy as np
    if cold:
        scrub = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        scrub2 = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = []
    for _ in range(n):
        if cold:
            scrub.fill_(1)
            scrub2.sum()
        else:
            run()
        e0.record(stream)
        run()
        e1.record(stream)
        torch.cuda.synchronize()
        t.append(e0.elapsed_time(e1) * 1e3)
    return float(np.median(t)), float(min(t))


def volume_sweep(w, ctx, stream, torch, ls, U, sizes=(8, 12, 16, 20, 24, 28, 32), shapes=None):
    """FP32 12-real EO dslash on L^3 x 2L lattices (or the given X x Y x Z x T shapes):
    warm (5 x 100 back-to-back launches, median and minimum) and single launches timed
    alone, warm and cold (after 1 GiB of other traffic).  The links are the sub-box of the
    32^3 x 64 field: i.i.d. per link, so each is a field of the same distribution."""
    import numpy as np
    rows = []
    for dims in (shapes if shapes is not None else [(L, L, L, 2 * L) for L in sizes]):
        X, Y, Z, T = dims
        Vh = X * Y * Z * T // 2
        if T > U.shape[1] or Z > U.shape[2] or Y > U.shape[3] or X > U.shape[4]:
            continue
        g = w.Gauge(ctx, dims, BC, w.RECON_12)
        g.upload(np.ascontiguousarray(U[:, :T, :Z, :Y, :X]))
        g.prepare(w.F32)
        lat = w.lattice(dims, BC)
        fin = w.pack(ctx, lat, w.ODD, w.F32, ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2, X), ls.STREAM_SPINOR))
        fout = w.new_field(lat, w.EVEN, w.F32)
        if shapes is None or w.tune_get(ctx, w.dslash_key(dims, w.F32, 12, 1, 0, 0)) is None:
            w.wd_autotune_dslash(g.handle, w.F32, 1, None)   # (a loaded tuning table is kept)
        run = lambda: w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fout.data_ptr())
        med, mn = timed_repeats(run, stream, torch)
        ws = Vh * BYTES_DSLASH
        row = {"lattice": "%dx%dx%dx%d" % dims, "even_sites": Vh, "working_set_mb": round(ws / 1e6, 1),
               "warm_us_median": round(med, 3), "warm_us_min": round(mn, 3),
               "warm_gflops": round(Vh * FLOPS_DSLASH / med / 1e3, 1),
               "warm_frac_hbm": round(ws / med / 1e3 / HBM_PEAK_GBS, 4),
               "tuned": w.tune_get(ctx, w.dslash_key(dims, w.F32, 12, 1, 0, 0))}
        if shapes is None:
            row["L"] = X
            for mode, cold in (("warm_single", False), ("cold", True)):
                med1, mn1 = single_launch_us(run, stream, torch, cold)
                row.update({mode + "_us_median": round(med1, 3), mode + "_us_min": round(mn1, 3)})
            row.update({"cold_gflops": round(Vh * FLOPS_DSLASH / row["cold_us_median"] / 1e3, 1),
                        "cold_frac_hbm": round(ws / row["cold_us_median"] / 1e3 / HBM_PEAK_GBS, 4)})
        rows.append(row)
        del fin, fout
        g.close()
    return {"kernel": "dslash_kernel<F32, r12>, autotuned per lattice", "bytes_per_site": BYTES_DSLASH, "rows": rows}


def slab_extras(w, ctx, stream, torch, ls, U, nslab=8, link_gbs=153.0):
    """One device's share of the 32^3 x 64 lattice split into `nslab` t-slabs: the
    slab dslash with half-spinor faces (F32, 12-real links) against the ordinary
    dslash on the same slab, the face packing, and the bytes each face sends.
    The transfer time is modelled at one inter-device link per face direction
    (about 153 GB/s each); on one device the faces are copies of its own."""
    import numpy as np
    X, Y, Z, T = DIMS
    Tl = T // nslab
    dims = (X, Y, Z, Tl)
    Vh = X * Y * Z * Tl // 2
    g = w.Gauge(ctx, dims, BC, w.RECON_12)
    g.upload(np.ascontiguousarray(U[:, :Tl]))
    g.prepare(w.F32)
    lat = w.lattice(dims, BC)
    fin = w.pack(ctx, lat, w.ODD, w.F32, ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2, 99), ls.STREAM_SPINOR))
    fout = w.new_field(lat, w.EVEN, w.F32)
    ff, fb = w.new_face(lat, w.F32), w.new_face(lat, w.F32)
    gf, gb = w.new_face(lat, w.F32), w.new_face(lat, w.F32)
    w.wd_halo_pack(g.handle, w.ODD, 0, w.F32, fin.data_ptr(), gf.data_ptr(), gb.data_ptr())
    w.wd_autotune_dslash(g.handle, w.F32, 1, None)
    pack_us, _ = timed_repeats(lambda: w.wd_halo_pack(g.handle, w.ODD, 0, w.F32, fin.data_ptr(), ff.data_ptr(),
                                                      fb.data_ptr()), stream, torch)
    halo_us, _ = timed_repeats(lambda: w.wd_dslash_halo(g.handle, w.EVEN, 0, w.F32, fin.data_ptr(), gf.data_ptr(),
                                                        gb.data_ptr(), 1.0, 1.0, fout.data_ptr()), stream, torch)
    plain_us, _ = timed_repeats(lambda: w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fout.data_ptr()),
                                stream, torch)
    face = w.face_bytes(lat, w.F32)
    g.close()
    return {"slab": "%dx%dx%dx%d" % dims, "of": "%dx%dx%dx%d" % DIMS, "slabs": nslab, "even_sites": Vh,
            "us_dslash_with_faces": round(halo_us, 3), "us_dslash_periodic_slab": round(plain_us, 3),
            "us_pack_both_faces": round(pack_us, 3),
            "gflops_with_faces": round(Vh * FLOPS_DSLASH / halo_us / 1e3, 1),
            "face_bytes_per_direction": face, "face_bytes_full_spinor_would_be": 2 * face,
            "modelled_transfer_us_per_direction": round(face / (link_gbs * 1e3), 2)}


def multi_rhs_records(w, ctx, ls, timed):
    """16 rhs on 16^3 x 32, FP32 and BF16, tuned: one launch against one launch per rhs, and
    for BF16 the matrix-core path against the per-rhs kernel."""
    out = {}
    dims, nrhs = (16, 16, 16, 32), 16
    Vh = 16 * 16 * 16 * 32 // 2
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(ls.gauge_field(dims, 0.5, ls.link_seed(4)))
    lat = w.lattice(dims, BC)
    psi = ls.gaussian_complex((nrhs, Vh, 4, 3), ls.source_seed(4), ls.STREAM_SPINOR)
    for prec in (w.F32, w.BF16):
        name = w.PREC_NAMES[prec]
        fin = w.pack(ctx, lat, w.ODD, prec, psi, nrhs)
        fout = w.new_field(lat, w.EVEN, prec, nrhs)
        w.wd_autotune_dslash(g.handle, prec, nrhs, None)
        us = timed(lambda: w.wd_dslash(g.handle, w.EVEN, 0, prec, nrhs, fin.data_ptr(), fout.data_ptr()), 50)
        # separate launches per rhs, for comparison
        hb = w.spinor_bytes(lat, w.EVEN, prec)
        us1 = timed(lambda: [w.wd_dslash(g.handle, w.EVEN, 0, prec, 1, fin.data_ptr() + r * hb, fout.data_ptr() + r * hb)
                             for r in range(nrhs)], 10)
        rec = {"nrhs": nrhs, "us_per_call": round(us, 2), "gflops": round(nrhs * Vh * FLOPS_DSLASH / us / 1e3, 1),
               "us_one_rhs_per_launch": round(us1, 2), "tuned": w.tune_get(ctx, w.dslash_key(dims, prec, 12, nrhs, 0, 0))}
        if prec != w.F32:
            # the colour multiply of 16 rhs on the matrix cores against the per-rhs kernel
            for flag, key in (("1", "us_matrix_core_path"), ("0", "us_per_rhs_path")):
                os.environ["WD_DSLASH_MFMA"] = flag
                rec[key] = round(timed(lambda: w.wd_dslash(g.handle, w.EVEN, 0, prec, nrhs, fin.data_ptr(),
                                                           fout.data_ptr()), 50), 2)
            del os.environ["WD_DSLASH_MFMA"]
        out["multi_rhs_16c32_%s" % name] = rec
    g.close()
    return out


def extras(w, ctx, stream, torch, ls, multi_rhs_only=False):
    """Multi-rhs (16 rhs on 16^3 x 32) and the ragged batch (8^4, 12^4, 16^3 x 32,
    24^3 x 32 in one persistent graph launch): time per call and GFLOP/s."""
    import ctypes
    out = {}

    def timed(fn, n):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / n

    out.update(multi_rhs_records(w, ctx, ls, timed))
    if multi_rhs_only:
        return out

    # the ragged lattices alone, then together with the 16-rhs item in the same single launch
    ragged = [((8, 8, 8, 8), 1), ((12, 12, 12, 12), 1), ((16, 16, 16, 32), 1), ((24, 24, 24, 32), 1)]
    for name, specs in (("ragged_batch", ragged), ("multi_rhs_and_ragged_one_launch", [((16, 16, 16, 32), 16)] + ragged)):
        for prec in (w.F32, w.BF16):
            items = (w.WdBatchItem * len(specs))()
            keep = []
            sites = site_rhs = nbytes = 0
            link_b, spin_b = (48, 96) if prec == w.F32 else (24, 52)
            for i, (d, nr) in enumerate(specs):
                gi = w.Gauge(ctx, d, BC, 12)
                seed = ls.link_seed(4, i + 1) if nr == 1 else ls.link_seed(4)
                gi.upload(ls.gauge_field(d, 0.5, seed))
                li = w.lattice(d, BC)
                vh = d[0] * d[1] * d[2] * d[3] // 2
                src = ls.gaussian_complex((nr, vh, 4, 3), ls.source_seed(4, i + 1) if nr == 1 else ls.source_seed(4),
                                          ls.STREAM_SPINOR)
                fi = w.pack(ctx, li, w.ODD, prec, src, nr)
                fo = w.new_field(li, w.EVEN, prec, nr)
                items[i].gauge, items[i].out_subset, items[i].dagger, items[i].nrhs = gi.handle.value, w.EVEN, 0, nr
                items[i].in_, items[i].out = fi.data_ptr(), fo.data_ptr()
                keep.append((gi, fi, fo))
                sites += vh
                site_rhs += vh * nr
                nbytes += vh * 8 * link_b + vh * nr * 2 * spin_b   # links once per site, spinors per rhs
            b = ctypes.c_void_p()
            w.wd_batch_create(ctx.handle, len(specs), items, prec, ctypes.byref(b))
            us = timed(lambda: w.wd_batch_run(b), 50)
            blk, wpc, pf = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            w.wd_batch_shape(b, ctypes.byref(blk), ctypes.byref(wpc), ctypes.byref(pf))
            nt, grid = ctypes.c_longlong(), ctypes.c_int()
            w.wd_batch_info(b, ctypes.byref(nt), ctypes.byref(grid))
            w.wd_batch_destroy(b)
            out["%s_%s" % (name, w.PREC_NAMES[prec])] = {
                "items": ["%dx%dx%dx%d x %d rhs" % (d + (nr,)) for d, nr in specs], "even_sites": sites,
                "site_rhs": site_rhs, "launches_per_call": 1, "us_per_call": round(us, 2),
                "gflops": round(site_rhs * FLOPS_DSLASH / us / 1e3, 1), "algorithmic_mb": round(nbytes / 1e6, 1),
                "gbs_algorithmic": round(nbytes / us / 1e3, 1), "frac_hbm": round(nbytes / us / 1e3 / HBM_PEAK_GBS, 4),
                "tiles": nt.value, "persistent_workgroups": grid.value,
                "tuned_shape": {"tile_sites": blk.value, "waves_per_cu": wpc.value, "pf": pf.value}}
            for gi, _, _ in keep:
                gi.close()
    return out


def solve_extras(w, ctx, torch, ls, dims=(32, 32, 32, 64), eps=0.6, kappa=0.1245, tol=1e-10, mdagm_gflops=None):
    """Time to an FP64-verified 1e-10 Wilson-system residual on 32^3 x 64 (eps 0.6,
    kappa 0.1245) through the even-odd CG, per inner (sloppy) storage precision,
    the level where pure FP32 recurrences stall, and flexible GMRES on the Schur
    complement without and with the learned preconditioner."""
    import ctypes
    X, Y, Z, T = dims
    g = w.Gauge(ctx, dims, BC, 12)
    U = ls.gauge_field(dims, eps, ls.link_seed(3))
    g.upload(U)
    lat = w.lattice(dims, BC)
    b = ls.gaussian_complex((T, Z, Y, X, 4, 3), ls.source_seed(3), ls.STREAM_SPINOR)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    for p in (w.F64, w.F32, w.F16, w.BF16):
        g.prepare(p)
        w.wd_autotune_dslash(g.handle, p, 1, None)
    out = {"lattice": list(dims), "eps": eps, "kappa": kappa, "tol": tol, "plaquette": round(plaquette(U), 6)}
    del U
    Vh = X * Y * Z * T // 2

    def rates(d):
        # operator flops only (the BLAS is not counted), per second of the whole solve: every
        # hopping-term application the solve queued (FP64 ones included), each with half a fused
        # update, so that four make one Mhat^dag Mhat as the bench step counts it
        gf = d["hops"] * Vh * (FLOPS_DSLASH + FLOPS_XPAY / 2) / d["seconds"] / 1e9
        d["operator_gflops"] = round(gf, 1)
        if mdagm_gflops:
            d["operator_gflops_over_mdagm_kernel"] = round(gf / mdagm_gflops, 3)
    runs = [("f64", w.F64, False), ("f32", w.F32, False), ("f16", w.F16, False), ("bf16", w.BF16, False),
            ("pure_f32", w.F32, True)]
    default_delta = {w.F32: 1e-5, w.F16: 1e-2, w.BF16: 3e-2}   # the library's defaults (delta < 0)
    for name, p, pure in runs:
        secs = []
        for rep in range(2):   # the first solve of a precision also sizes the workspace
            fx = torch.zeros_like(fb)
            prm = w.solver_params(tol=tol, maxiter=5000, sloppy=p, delta=-1.0, pure_sloppy=pure)
            info = w.WdSolverInfo()
            w.wd_wilson_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info),
                              ok=(w.WD_OK, w.WD_ENOCONV))
            secs.append(info.seconds)
        d = {k: v for k, v in info.as_dict().items() if k not in ("cycles", "fell_back")}
        d["cond_estimate"] = round(d["lambda_max"] / d["lambda_min"], 3) if d["lambda_min"] > 0 else None
        rates(d)
        d["seconds"] = round(d["seconds"], 5)
        d["seconds_first"] = round(secs[0], 5)
        d["delta"] = None if (pure or p == w.F64) else default_delta[p]
        out[name] = d
    # BiCGstab on the Schur complement (FP32 iterations, FP64 reliable updates)
    for name, p in (("bicgstab_f32", w.F32), ("bicgstab_f16", w.F16), ("bicgstab_bf16", w.BF16)):
        secs = []
        for rep in range(2):
            fx = torch.zeros_like(fb)
            prm = w.solver_params(tol=tol, maxiter=5000, sloppy=p, delta=-1.0)
            info = w.WdSolverInfo()
            w.wd_bicgstab_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info),
                                ok=(w.WD_OK, w.WD_ENOCONV))
            secs.append(info.seconds)
        d = {k: v for k, v in info.as_dict().items() if k not in ("cycles", "fell_back", "lambda_min", "lambda_max")}
        rates(d)
        d["seconds"] = round(d["seconds"], 5)
        d["seconds_first"] = round(secs[0], 5)
        out[name] = d
    # flexible GMRES on the Schur complement (FP32 cycles, FP64 refinement), without and with
    # the network trained on 16^3 x 32 (applied here as trained: the layer is local)
    from paper_0810_5365_amd import learn
    net = learn.load_net(learn.DEFAULT_WEIGHTS, w.BF16)
    ws = net.storage()
    wid = (ctypes.c_int * len(net.widths))(*net.widths)
    ptrs = (ctypes.c_void_p * len(ws))(*[t.data_ptr() for t in ws])
    for name, nl in (("fgmres_f32", 0), ("fgmres_learned_f32", len(ws))):
        secs = []
        for rep in range(2):
            fx = torch.zeros_like(fb)
            prm = w.solver_params(tol=tol, maxiter=2000, sloppy=w.F32, delta=-1.0)   # library default (1e-5)
            info = w.WdSolverInfo()
            w.wd_fgmres_solve(g.handle, kappa, ctypes.byref(prm), 16, nl, wid if nl else None, ptrs if nl else None,
                              net.wprec, fb.data_ptr(), fx.data_ptr(), ctypes.byref(info), ok=(w.WD_OK, w.WD_ENOCONV))
            secs.append(info.seconds)
        d = {k: v for k, v in info.as_dict().items() if k not in ("lambda_min", "lambda_max")}
        rates(d)
        d["seconds"] = round(d["seconds"], 5)
        d["seconds_first"] = round(secs[0], 5)
        d["restart"], d["delta"] = 16, 1e-5
        out[name] = d
    g.close()
    out["network_apply_even"] = network_apply_times(w, ctx, net, dims, reps=20)
    return out


def network_layer_times(w, ctx, net, dims, reps=100):
    """Each layer of the committed network (bf16 weights, matrix-core mixing) on random
    features over the whole lattice: microseconds per launch (HIP events on the stream)."""
    import torch
    import lattice_synth as ls
    f = __import__("paper_0810_5365_amd.learn", fromlist=["Field"]).Field(ctx, dims, 0.7, 6001)
    stream = torch.cuda.current_stream(0)
    V = dims[0] * dims[1] * dims[2] * dims[3]
    gen = torch.Generator().manual_seed(7)
    res = {}
    for (cin, cout), Ws in zip(zip(net.widths[:-1], net.widths[1:]), net.storage()):
        x = torch.randn(cin * 6 * V, generator=gen).cuda()
        y = torch.empty(cout * 6 * V, device="cuda")
        run = lambda: w.wd_ptconv_forward(f.g.handle, cin, cout, net.wprec, 1, Ws.data_ptr(), x.data_ptr(), y.data_ptr())
        for _ in range(5):
            run()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        res["%d->%d" % (cin, cout)] = round(e0.elapsed_time(e1) * 1e3 / reps, 2)
    f.close()
    return {"lattice": list(dims), "us_per_launch": res,
            "unique_bytes_per_site": {k: (int(k.split("->")[0]) + int(k.split("->")[1])) * 24 + 4 * 48 for k in res}}


def network_apply_times(w, ctx, net, dims, reps=100):
    """The preconditioner as the learned solve applies it (the even sites of N (v_e, 0)), with
    the hidden features in bf16 (the default) and in float32: microseconds per application."""
    import ctypes
    import os
    import torch
    import lattice_synth as ls
    f = __import__("paper_0810_5365_amd.learn", fromlist=["Field"]).Field(ctx, dims, 0.7, 6001)
    stream = torch.cuda.current_stream(0)
    lat = w.lattice(dims, BC)
    Vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    fin = w.pack(ctx, lat, w.EVEN, w.F32, ls.gaussian_complex((Vh, 4, 3), 17, ls.STREAM_SPINOR))
    fout = w.new_field(lat, w.EVEN, w.F32)
    ws = net.storage()
    widths = (ctypes.c_int * len(net.widths))(*net.widths)
    ptrs = (ctypes.c_void_p * len(ws))(*[t.data_ptr() for t in ws])
    run = lambda: w.wd_ptnet_apply_even(f.g.handle, len(ws), widths, ptrs, net.wprec, fin.data_ptr(), fout.data_ptr())
    res = {}
    for mode, env in (("bf16_hidden", {}), ("bf16_hidden_unsplit", {"WD_PTCONV_SPLIT": "0"}),
                      ("f32_hidden", {"WD_PTNET_F32_FEATURES": "1"})):
        os.environ.update(env)
        med, mn = timed_repeats(run, stream, torch, n=reps)
        for k in env:
            os.environ.pop(k, None)
        res[mode] = {"us_median": round(med, 2), "us_min": round(mn, 2)}
    f.close()
    return {"lattice": list(dims), "widths": list(net.widths), **res}


def learned_extras(w, ctx):
    """Time to an FP64-verified 1e-10 Wilson-system residual on 16^3 x 32 (eps 0.7, kappa 0.1248),
    four gauge fields unseen in training: plain FP32 CG (with FP64 reliable updates), flexible
    GMRES without and with the committed trained network (bf16 weights on the matrix cores)."""
    import numpy as np
    import lattice_synth as ls
    from paper_0810_5365_amd import learn
    net = learn.load_net(learn.DEFAULT_WEIGHTS, w.BF16)
    dims, kappa = (16, 16, 16, 32), 0.1248
    rows = []
    for seed in (6001, 6002, 6003, 6004):
        f = learn.Field(ctx, dims, 0.7, seed)
        learn.solve_compare(net, f, kappa)          # first call: packing, tuning-free warm-up
        r = learn.solve_compare(net, f, kappa)
        row = {k: {kk: v[kk] for kk in ("iters", "wall_s", "true_resid_M", "fell_back")}
               for k, v in r.items() if isinstance(v, dict)}
        cg = r["plain_cg_f32"]
        row["field"] = {"seed": seed, "plaquette": round(plaquette(ls.gauge_field(dims, 0.7, seed)), 6),
                        "lambda_min_mdagm": cg["lambda_min"], "lambda_max_mdagm": cg["lambda_max"],
                        "cond_mdagm": round(cg["lambda_max"] / cg["lambda_min"], 3) if cg["lambda_min"] > 0 else None}
        rows.append(row)
        f.close()
    out = {"lattice": list(dims), "eps": 0.7, "kappa": kappa, "tol": 1e-10, "fields": [6001, 6002, 6003, 6004],
           "weights": "paper_0810_5365_amd/data/" + __import__("os").path.basename(learn.DEFAULT_WEIGHTS), "per_field": rows}
    for k in (k for k in rows[0] if k != "field"):
        out["mean_" + k] = {"iters": float(np.mean([r[k]["iters"] for r in rows])),
                            "wall_ms": round(1e3 * float(np.mean([r[k]["wall_s"] for r in rows])), 3)}
    out["learned_speedup_vs_plain_cg"] = round(out["mean_plain_cg_f32"]["wall_ms"] / out["mean_fgmres_learned"]["wall_ms"], 3)
    out["network_layers"] = network_layer_times(w, ctx, net, dims)
    out["network_apply_even"] = network_apply_times(w, ctx, net, dims)
    out["learned_speedup_vs_fgmres_no_net"] = round(out["mean_fgmres_no_net"]["wall_ms"] / out["mean_fgmres_learned"]["wall_ms"], 3)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import lattice_synth as ls
    from paper_0810_5365_amd import wdirac as w

    dims = tuple(args.dims)
    X, Y, Z, T = dims
    Vh = X * Y * Z * T // 2
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(0)
    ctx = w.Context(0, stream.cuda_stream)
    def copy_reference():
        # a 2 GiB copy (read and write), the reference for hardware byte counters in the same run
        src = torch.ones(1 << 31, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            w.wd_device_copy(ctx.handle, src.data_ptr(), dst.data_ptr(), 1 << 31)
        torch.cuda.synchronize()
        del src, dst

    if args.multi_rhs_only:
        rec = extras(w, ctx, stream, torch, ls, multi_rhs_only=True)
        copy_reference()
        print(json.dumps({"multi_rhs": rec}), flush=True)
        ctx.close()
        return
    if args.network_only:
        from paper_0810_5365_amd import learn
        net = learn.load_net(learn.DEFAULT_WEIGHTS, w.BF16)
        rec = {"x".join(map(str, d)): network_apply_times(w, ctx, net, d) for d in ((32, 32, 32, 64), (16, 16, 16, 32))}
        copy_reference()
        print(json.dumps({"network_apply_even": rec}), flush=True)
        ctx.close()
        return

    print("bench: generating %s links and source" % (dims,), file=sys.stderr, flush=True)
    U = ls.gauge_field(dims, EPS, ls.link_seed(2))
    psi_e = ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2), ls.STREAM_SPINOR)
    if args.shape_sweep_only:
        # with --tune-cache: the launch shapes of an earlier run are loaded (so that a counter run
        # under a profiler times the same configurations), else tuned and saved there
        have = bool(args.tune_cache) and os.path.exists(args.tune_cache)
        if have:
            w.wd_tune_load(ctx.handle, args.tune_cache.encode())
        sweep = volume_sweep(w, ctx, stream, torch, ls, U, shapes=SHAPE_SWEEP)
        if args.tune_cache and not have:
            w.wd_tune_save(ctx.handle, args.tune_cache.encode())
        print(json.dumps({"shape_sweep": sweep}), flush=True)
        ctx.close()
        return
    g = w.Gauge(ctx, dims, BC, w.RECON_12)
    g.upload(U)
    if args.precision_sweep_only:
        # with --tune-cache: the launch shapes of an earlier run are loaded (so that counter runs
        # under a profiler time the same configurations), else tuned and saved there
        have = bool(args.tune_cache) and os.path.exists(args.tune_cache)
        if have:
            w.wd_tune_load(ctx.handle, args.tune_cache.encode())
        rec = dslash_by_precision(w, ctx, stream, torch, ls, g, dims,
                                  ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2, 1), ls.STREAM_SPINOR), U,
                                  tune=not have)
        if args.tune_cache and not have:
            w.wd_tune_save(ctx.handle, args.tune_cache.encode())
        print(json.dumps({"dslash_eo_by_precision": rec}), flush=True)
        g.close()
        ctx.close()
        return
    g.prepare(w.F32)
    lat = w.lattice(dims, BC)
    fin = w.pack(ctx, lat, w.EVEN, w.F32, psi_e)
    fout = w.new_field(lat, w.EVEN, w.F32)
    torch.cuda.synchronize()
    tuned = {}
    if args.tune_cache and os.path.exists(args.tune_cache):
        w.wd_tune_load(ctx.handle, args.tune_cache.encode())
    elif not args.no_tune:
        print("bench: autotuning the dslash launch shape", file=sys.stderr, flush=True)
        w.wd_autotune_dslash(g.handle, w.F32, 1, args.tune_cache.encode() if args.tune_cache else None)
    for dag in (0, 1):
        for xp in (0, 1):
            tuned["d%d_x%d" % (dag, xp)] = w.tune_get(ctx, w.dslash_key(dims, w.F32, 12, 1, dag, xp))

    def step():
        w.wd_apply_MdagM(g.handle, KAPPA, w.EVEN, w.F32, 1, fin.data_ptr(), fout.data_ptr())

    print("bench: warmup %d, timed %d steps" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    # the step's output, for the comparison with the oracle (before anything else writes fout)
    step_out = None if args.no_cpu else w.unpack(ctx, lat, w.EVEN, w.F32, fout, psi_e.shape)

    # the plain even-odd dslash D_eo alone (no fused update), same timing method
    fodd = w.new_field(lat, w.ODD, w.F32)
    fodd.zero_()
    for _ in range(5):
        w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n_eo = max(args.steps, 20)
    e0.record(stream)
    for _ in range(n_eo):
        w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    eo_us = e0.elapsed_time(e1) * 1e3 / n_eo
    eo_med, eo_min = timed_repeats(lambda: w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr()),
                                   stream, torch)
    eo_run = lambda: w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr())
    cold_med, cold_min = single_launch_us(eo_run, stream, torch, cold=True)
    eo = {"us_per_launch": round(eo_us, 3), "us_median_5x100": round(eo_med, 3), "us_min_5x100": round(eo_min, 3),
          "timing": "warm: back-to-back repeats on the same buffers (the 256 MB last-level cache keeps part "
                    "of the 604 MB working set between repeats); cold: one launch after 1 GiB of other traffic",
          "gflops": round(Vh * FLOPS_DSLASH / eo_us / 1e3, 1),
          "gbs_algorithmic": round(Vh * BYTES_DSLASH / eo_us / 1e3, 1),
          "frac_hbm": round(Vh * BYTES_DSLASH / eo_us / 1e3 / HBM_PEAK_GBS, 4),
          "cold_us_median": round(cold_med, 3), "cold_us_min": round(cold_min, 3),
          "cold_frac_hbm": round(Vh * BYTES_DSLASH / cold_med / 1e3 / HBM_PEAK_GBS, 4),
          "gbs_naive_no_reuse": round(Vh * (8 * (48 + 96) + 96) / eo_us / 1e3, 1)}

    by_prec = None
    if not args.no_extras:
        print("bench: EO dslash at every storage precision", file=sys.stderr, flush=True)
        by_prec = dslash_by_precision(w, ctx, stream, torch, ls, g, dims,
                                      ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2, 1), ls.STREAM_SPINOR), U)

    # achievable ceiling: streaming copy of 2 GiB (read + write bytes counted)
    nbytes = 2 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        w.wd_device_copy(ctx.handle, src.data_ptr(), dst.data_ptr(), nbytes)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        w.wd_device_copy(ctx.handle, src.data_ptr(), dst.data_ptr(), nbytes)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * nbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    # the paper's temporal-gauge trick on the same field: unit t-links on all but the last slice
    gf = None
    if not args.no_extras:
        print("bench: temporal gauge fixing", file=sys.stderr, flush=True)
        w.wd_gauge_fix_temporal(g.handle, None)
        for _ in range(5):
            w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr())
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n_eo):
            w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fodd.data_ptr(), fout.data_ptr())
        e1.record(stream)
        torch.cuda.synchronize()
        gf_us = e0.elapsed_time(e1) * 1e3 / n_eo
        gf_bytes = BYTES_DSLASH - 2 * 48 * (dims[3] - 1) / dims[3]   # t-links read on one slice only
        gf = {"us_per_launch": round(gf_us, 3), "gflops_effective": round(Vh * FLOPS_DSLASH / gf_us / 1e3, 1),
              "bytes_per_site": round(gf_bytes, 2), "gbs_algorithmic": round(Vh * gf_bytes / gf_us / 1e3, 1),
              "speedup_vs_plain": round(eo_us / gf_us, 3)}

    flops_step = Vh * 2 * (2 * FLOPS_DSLASH + FLOPS_XPAY)
    gflops = flops_step / (ms_per_step * 1e-3) / 1e9
    # the timed region holds only dslash launches: 4 per step, 2 of them with the fused xpay
    launches = 4 * args.steps
    avg_launch_s = ms * 1e-3 / launches
    bytes_per_launch = Vh * (BYTES_DSLASH + BYTES_XPAY / 2.0)   # averaged over the 4 launches
    achieved = bytes_per_launch / avg_launch_s / 1e9

    traffic = measured_traffic(dims)

    rec = {
        "metric": "dslash GFLOP/s & %HBM roofline; time to 1e-10 solve, plain vs mixed+learned",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: SU(3) links exp(i*0.5*H) reunitarised, Gaussian source (seeded Philox)",
        "config": {"workload": "Mhat^dag Mhat (even-odd Wilson, 4 dslash/step), %dx%dx%dx%d, FP32, 12-real links, "
                               "kappa=%g, bc=(+,+,+,-)" % (*dims, KAPPA),
                   "lattice": list(dims), "even_sites": Vh, "flops_per_step": flops_step},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "dslash_kernel<F32, r12> (4 launches/step, 2 with xpay)",
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_launch_s * 1e6, 3)},
        "wall_s_timed": round(wall, 4),
        "dslash_eo": eo,
        "dslash_eo_temporal_gauge": gf,
        "dslash_eo_by_precision": by_prec,
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
        "tuned_launch": tuned,
        # the paper's own figures (Section 1 and Section 7), on other hardware: context only
        "context_paper_gflops": {"wilson_dslash_tesla_c870": 68, "wilson_dslash_gtx_280": 92,
                                 "eo_operator_tesla_c870": ">60", "eo_operator_gtx_280": "~90",
                                 "cg_tesla_c870": ">50", "cg_gtx_280": ">80", "sse_cpu_xeon": "<5"},
    }
    if not args.no_extras:
        print("bench: multi-rhs and ragged-batch measurements", file=sys.stderr, flush=True)
        rec["extras"] = extras(w, ctx, stream, torch, ls)
        print("bench: 32^3x64 solves", file=sys.stderr, flush=True)
        rec["solve_32c64"] = solve_extras(w, ctx, torch, ls, mdagm_gflops=gflops)
        print("bench: learned vs plain solves on 16^3x32", file=sys.stderr, flush=True)
        rec["solve_learned_16c32"] = learned_extras(w, ctx)
    if not args.no_extras and not args.no_sweep and dims == DIMS:
        print("bench: volume sweep L^3 x 2L", file=sys.stderr, flush=True)
        rec["volume_sweep"] = volume_sweep(w, ctx, stream, torch, ls, U)
        print("bench: lattices one extent short of 32^3 x 64", file=sys.stderr, flush=True)
        rec["shape_sweep"] = volume_sweep(w, ctx, stream, torch, ls, U, shapes=SHAPE_SWEEP)
        print("bench: one t-slab of eight with half-spinor faces", file=sys.stderr, flush=True)
        rec["slab_32c8_of_32c64"] = slab_extras(w, ctx, stream, torch, ls, U)
    if not args.no_cpu:
        print("bench: timing the CPU oracle baseline", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(U, psi_e, dims, step_out)
        rec["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(rec), flush=True)
    g.close()
    ctx.close()


if __name__ == "__main__":
    main()
