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

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
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
    return ap.parse_args()


def cpu_baseline(U, psi_e, dims):
    """The FP64 oracle's Mhat^dagger Mhat on the same inputs (one application)."""
    import oracle as orc
    Vh = psi_e.shape[0]
    orc.parity_sites(dims, 0)
    orc.parity_sites(dims, 1)   # build the checkerboard index tables outside the timing
    t0 = time.perf_counter()
    reps = 0
    while True:
        orc.mhat_dag_mhat(U, psi_e, KAPPA, BC)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 3:
            break
    dt = (time.perf_counter() - t0) / reps
    flops = Vh * 2 * (2 * FLOPS_DSLASH + FLOPS_XPAY)
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": "%d application(s) of the FP64 oracle's Mhat^dag Mhat on the full %dx%dx%dx%d lattice "
                      "(%d even sites), %.2f s each" % (reps, *dims, Vh, dt)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
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

    print("bench: generating %s links and source" % (dims,), file=sys.stderr, flush=True)
    U = ls.gauge_field(dims, EPS, ls.link_seed(2))
    psi_e = ls.gaussian_complex((Vh, 4, 3), ls.source_seed(2), ls.STREAM_SPINOR)
    g = w.Gauge(ctx, dims, BC, w.RECON_12)
    g.upload(U)
    g.prepare(w.F32)
    lat = w.lattice(dims, BC)
    fin = w.pack(ctx, lat, w.EVEN, w.F32, psi_e)
    fout = w.new_field(lat, w.EVEN, w.F32)
    torch.cuda.synchronize()

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

    flops_step = Vh * 2 * (2 * FLOPS_DSLASH + FLOPS_XPAY)
    gflops = flops_step / (ms_per_step * 1e-3) / 1e9
    # the timed region holds only dslash launches: 4 per step, 2 of them with the fused xpay
    launches = 4 * args.steps
    avg_launch_s = ms * 1e-3 / launches
    bytes_per_launch = Vh * (BYTES_DSLASH + BYTES_XPAY / 2.0)   # averaged over the 4 launches
    achieved = bytes_per_launch / avg_launch_s / 1e9

    traffic = None
    tr_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "dslash_f32_r12_32c64_traffic.json")
    if os.path.exists(tr_path):
        try:
            traffic = json.load(open(tr_path)).get("bytes_per_launch")
        except Exception:
            traffic = None

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
    }
    if not args.no_cpu:
        print("bench: timing the CPU oracle baseline", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(U, psi_e, dims)
        rec["cpu_baseline"]["host"] = platform.processor() or platform.machine()
    print(json.dumps(rec), flush=True)
    g.close()
    ctx.close()


if __name__ == "__main__":
    main()
