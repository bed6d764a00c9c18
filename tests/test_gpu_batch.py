"""GPU: many right-hand sides and a ragged batch of lattices in one persistent
launch replayed from a hipGraph, each lattice and each rhs checked against the
FP64 oracle separately."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def w():
    from paper_0810_5365_amd import wdirac
    return wdirac


def half_source(dims, seed, nrhs):
    X, Y, Z, T = dims
    return ls.gaussian_complex((nrhs, X * Y * Z * T // 2, 4, 3), seed, ls.STREAM_SPINOR)


def ref_hop(U, psi, out_subset_even, dagger):
    return orc.d_eo(U, psi, BC, dagger) if out_subset_even else orc.d_oe(U, psi, BC, dagger)


@pytest.mark.parametrize("rhs_inner", [0, 1])
def test_multi_rhs_orderings(w, monkeypatch, rhs_inner):
    monkeypatch.setenv("WD_DSLASH_RHS_INNER", str(rhs_inner))
    dims, nrhs = (6, 4, 10, 4), 5
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.5, 23)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    psi = half_source(dims, 9, nrhs)
    fin = w.pack(ctx, lat, w.EVEN, w.F32, psi, nrhs)
    fout = w.new_field(lat, w.ODD, w.F32, nrhs)
    w.wd_dslash(g.handle, w.ODD, 0, w.F32, nrhs, fin.data_ptr(), fout.data_ptr())
    got = w.unpack(ctx, lat, w.ODD, w.F32, fout, psi.shape, nrhs)
    ref = orc.d_oe(U, psi, BC)
    for r in range(nrhs):
        assert orc.rel_l2(got[r], ref[r]) < 1e-5
    g.close()
    ctx.close()


_INPUTS = {}


def _inputs(dims, seed, nrhs):
    """Seeded links (eps 0.5) and nrhs input half fields, generated once per module."""
    key = (dims, seed, nrhs)
    if key not in _INPUTS:
        _INPUTS[key] = (ls.gauge_field(dims, 0.5, seed), half_source(dims, seed + 1, nrhs))
    return _INPUTS[key]


_REFS = {}


def _ref(spec):
    """The oracle's hopping term for one batch item (all its rhs), computed once per module."""
    if spec not in _REFS:
        dims, out_even, dagger, nrhs, seed = spec
        U, psi = _inputs(dims, seed, nrhs)
        _REFS[spec] = ref_hop(U, psi, out_even, bool(dagger))
    return _REFS[spec]


def _run_batch(w, ctx, specs, prec, replays=3):
    """specs: list of (dims, out_even, dagger, nrhs, seed)."""
    import torch
    items = (w.WdBatchItem * len(specs))()
    keep = []
    for i, (dims, out_even, dagger, nrhs, seed) in enumerate(specs):
        U, psi = _inputs(dims, seed, nrhs)
        g = w.Gauge(ctx, dims, BC, 12)
        g.upload(U)
        lat = w.lattice(dims, BC)
        in_sub, out_sub = (w.ODD, w.EVEN) if out_even else (w.EVEN, w.ODD)
        fin = w.pack(ctx, lat, in_sub, prec, psi, nrhs)
        fout = w.new_field(lat, out_sub, prec, nrhs)
        fout.zero_()
        items[i].gauge = g.handle.value
        items[i].out_subset = out_sub
        items[i].dagger = dagger
        items[i].nrhs = nrhs
        items[i].in_ = fin.data_ptr()
        items[i].out = fout.data_ptr()
        keep.append((U, g, lat, psi, fin, fout, out_sub, out_even, dagger, nrhs))
    b = ctypes.c_void_p()
    w.wd_batch_create(ctx.handle, len(specs), items, prec, ctypes.byref(b))
    nt, grid = ctypes.c_longlong(), ctypes.c_int()
    w.wd_batch_info(b, ctypes.byref(nt), ctypes.byref(grid))
    blk, wpc, pf = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    w.wd_batch_shape(b, ctypes.byref(blk), ctypes.byref(wpc), ctypes.byref(pf))
    results = []
    for rep in range(replays):
        for k in keep:
            k[5].zero_()                     # eager work between replays
        torch.cuda.synchronize()
        w.wd_batch_run(b)
        torch.cuda.synchronize()
        outs = [w.unpack(ctx, k[2], k[6], prec, k[5], k[3].shape, k[9]) for k in keep]
        results.append(outs)
    w.wd_batch_destroy(b)
    return keep, results, nt.value, grid.value, (blk.value, wpc.value, pf.value)


def test_ragged_batch_one_launch_f32(w):
    ctx = w.Context(0)
    specs = [((8, 8, 8, 8), True, 0, 3, 101), ((12, 12, 12, 12), False, 1, 1, 102),
             ((6, 4, 10, 4), True, 1, 2, 103), ((2, 2, 2, 2), False, 0, 1, 104)]
    keep, results, ntiles, grid, shape = _run_batch(w, ctx, specs, w.F32)
    blk, wpc, pf = shape   # the tuned launch shape
    assert blk in (64, 128, 256) and wpc in (8, 16, 24, 32) and pf in (0, 1)
    expect_tiles = sum(((d[0] * d[1] * d[2] * d[3] // 2 + blk - 1) // blk) * n for d, _, _, n, _ in specs)
    assert ntiles == expect_tiles and 1 <= grid <= ntiles
    for outs in results:
        for (U, g, lat, psi, fin, fout, out_sub, out_even, dagger, nrhs), got in zip(keep, outs):
            ref = ref_hop(U, psi, out_even, bool(dagger))
            for r in range(nrhs):
                assert orc.rel_l2(got[r], ref[r]) < 1e-5
    for k in keep:
        k[1].close()
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_ragged_batch_16bit(w, prec):
    ctx = w.Context(0)
    specs = [((8, 8, 8, 8), True, 0, 2, 201), ((12, 12, 12, 12), True, 0, 1, 202), ((4, 6, 2, 10), False, 1, 3, 203)]
    keep, results, _, _, _ = _run_batch(w, ctx, specs, w.PREC_BY_NAME[prec], replays=2)
    for outs in results:
        for (U, g, lat, psi, fin, fout, out_sub, out_even, dagger, nrhs), got in zip(keep, outs):
            ref = ref_hop(U, psi, out_even, bool(dagger))
            for r in range(nrhs):
                assert orc.rel_l2(got[r], ref[r]) < 5e-3
    for k in keep:
        k[1].close()
    ctx.close()


@pytest.mark.parametrize("block,waves,pf", [(64, 8, 0), (128, 32, 1), (256, 16, 1), (64, 24, 1)])
def test_ragged_batch_every_forced_shape(w, monkeypatch, block, waves, pf):
    """Launch shapes forced through the environment (no tuning): tile widths 64..256, waves
    per compute unit, pipelined directions; the tile count follows the width."""
    monkeypatch.setenv("WD_BATCH_BLOCK", str(block))
    monkeypatch.setenv("WD_BATCH_WAVES", str(waves))
    monkeypatch.setenv("WD_BATCH_PF", str(pf))
    ctx = w.Context(0)
    specs = [((8, 8, 8, 8), True, 0, 2, 301), ((6, 4, 10, 4), False, 1, 3, 302), ((2, 2, 2, 2), True, 1, 1, 303)]
    keep, results, ntiles, grid, shape = _run_batch(w, ctx, specs, w.F32, replays=2)
    assert shape == (block, waves, pf)
    assert ntiles == sum(((d[0] * d[1] * d[2] * d[3] // 2 + block - 1) // block) * n for d, _, _, n, _ in specs)
    assert 1 <= grid <= ntiles
    for outs in results:
        for (U, g, lat, psi, fin, fout, out_sub, out_even, dagger, nrhs), got in zip(keep, outs):
            ref = ref_hop(U, psi, out_even, bool(dagger))
            for r in range(nrhs):
                assert orc.rel_l2(got[r], ref[r]) < 1e-5
    for k in keep:
        k[1].close()
    ctx.close()


def test_batch_rejects_bad_items(w):
    ctx = w.Context(0)
    dims = (4, 4, 4, 4)
    g12 = w.Gauge(ctx, dims, BC, 12)
    g12.upload(ls.gauge_field(dims, 0.5, 1))
    g18 = w.Gauge(ctx, dims, BC, 18)
    g18.upload(ls.gauge_field(dims, 0.5, 1))
    lat = w.lattice(dims, BC)
    f = w.new_field(lat, w.EVEN, w.F32)
    items = (w.WdBatchItem * 2)()
    for i, g in enumerate((g12, g18)):
        items[i].gauge = g.handle.value
        items[i].out_subset = w.EVEN
        items[i].dagger = 0
        items[i].nrhs = 1
        items[i].in_ = f.data_ptr()
        items[i].out = f.data_ptr()
    b = ctypes.c_void_p()
    lib = w._raw()
    assert lib.wd_batch_create(ctx.handle, 2, items, w.F32, ctypes.byref(b)) == w.WD_EUNSUPPORTED
    items[1].gauge = g12.handle.value
    items[1].out_subset = w.FULL
    assert lib.wd_batch_create(ctx.handle, 2, items, w.F32, ctypes.byref(b)) == w.WD_EINVAL
    assert lib.wd_batch_create(ctx.handle, 0, items, w.F32, ctypes.byref(b)) == w.WD_EINVAL
    g12.close()
    g18.close()
    ctx.close()


def test_sixteen_rhs_on_16c32(w):
    """The multi-rhs workload at full size: 16 Gaussian right-hand sides on 16^3 x 32."""
    dims, nrhs = (16, 16, 16, 32), 16
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.5, ls.link_seed(4))
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    psi = half_source(dims, ls.source_seed(4), nrhs)
    ref = orc.d_eo(U, psi, BC)
    for prec, tol in ((w.F32, 1e-5), (w.BF16, 5e-3)):
        fin = w.pack(ctx, lat, w.ODD, prec, psi, nrhs)
        fout = w.new_field(lat, w.EVEN, prec, nrhs)
        w.wd_dslash(g.handle, w.EVEN, 0, prec, nrhs, fin.data_ptr(), fout.data_ptr())
        got = w.unpack(ctx, lat, w.EVEN, prec, fout, psi.shape, nrhs)
        for r in range(nrhs):
            assert orc.rel_l2(got[r], ref[r]) < tol
    g.close()
    ctx.close()


def test_ragged_batch_full_size_lattices(w):
    """The ragged workload at its real sizes: 8^4, 12^4, 16^3 x 32 and 24^3 x 32 in one launch."""
    ctx = w.Context(0)
    specs = [((8, 8, 8, 8), True, 0, 1, 4101), ((12, 12, 12, 12), True, 0, 1, 4102),
             ((16, 16, 16, 32), True, 0, 1, 4103), ((24, 24, 24, 32), True, 0, 1, 4104)]
    keep, results, _, _, _ = _run_batch(w, ctx, specs, w.F32, replays=2)
    for outs in results:
        for (U, g, lat, psi, fin, fout, out_sub, out_even, dagger, nrhs), got in zip(keep, outs):
            assert orc.rel_l2(got[0], ref_hop(U, psi, out_even, False)[0]) < 1e-5
    for k in keep:
        k[1].close()
    ctx.close()


# The multi-rhs and ragged workload as one batch: 16 Gaussian rhs on 16^3 x 32 together
# with the lattices 8^4, 12^4, 16^3 x 32 and 24^3 x 32 (eps 0.5), all in one launch.
C4_SPECS = [((16, 16, 16, 32), True, 0, 16, 4100), ((8, 8, 8, 8), True, 0, 1, 4101),
            ((12, 12, 12, 12), True, 0, 1, 4102), ((16, 16, 16, 32), True, 0, 1, 4103),
            ((24, 24, 24, 32), True, 0, 1, 4104)]
# two small items with ragged tiles, odd outputs and the dagger, appended for the forced shapes
SMALL_SPECS = [((2, 2, 2, 2), False, 1, 1, 4105), ((6, 4, 10, 4), False, 1, 3, 4106)]


def _site_max_err(got, ref):
    """Largest per-site error norm over the RMS site norm of the reference."""
    d = np.abs(got - ref).reshape(got.shape[0], -1)
    r = np.abs(ref).reshape(ref.shape[0], -1)
    return float(np.sqrt((d * d).sum(1)).max() / np.sqrt((r * r).sum(1).mean()))


def _check_items(keep, results, specs, tol, site_tol=None):
    for outs in results:
        for spec, k, got in zip(specs, keep, outs):
            ref = _ref(spec)
            for r in range(spec[3]):
                err = orc.rel_l2(got[r], ref[r])
                assert err < tol, (spec, r, err)
                if site_tol is not None:
                    assert _site_max_err(got[r], ref[r]) < site_tol, (spec, r)


@pytest.mark.parametrize("block,waves,pf", [(64, 1, 0), (128, 2, 0), (256, 1, 1)])
def test_persistent_batch_walks_many_tiles_per_workgroup(w, monkeypatch, block, waves, pf):
    """Forced launch shapes with far fewer persistent workgroups than tiles, so every
    workgroup walks a range of tiles across item boundaries: the full-size workload
    (16 rhs on 16^3 x 32 plus the four ragged lattices) and two small items with ragged
    tiles, odd outputs and the dagger, each rhs checked against the oracle."""
    monkeypatch.setenv("WD_BATCH_BLOCK", str(block))
    monkeypatch.setenv("WD_BATCH_WAVES", str(waves))
    monkeypatch.setenv("WD_BATCH_PF", str(pf))
    ctx = w.Context(0)
    specs = C4_SPECS + SMALL_SPECS
    keep, results, ntiles, grid, shape = _run_batch(w, ctx, specs, w.F32, replays=2)
    assert shape == (block, waves, pf)
    assert ntiles == sum(((d[0] * d[1] * d[2] * d[3] // 2 + block - 1) // block) * n for d, _, _, n, _ in specs)
    assert grid < ntiles and ntiles >= 20 * grid, (ntiles, grid)
    _check_items(keep, results, specs, 1e-5, site_tol=1e-5)
    for k in keep:
        k[1].close()
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_multi_rhs_and_ragged_lattices_in_one_launch(w, prec):
    """The 16-rhs item and the four ragged lattices in ONE batch (one graph launch), the
    launch shape autotuned: every rhs of every item against the oracle (F32 1e-5, BF16
    storage 5e-3)."""
    ctx = w.Context(0)
    p = w.PREC_BY_NAME[prec]
    keep, results, ntiles, grid, shape = _run_batch(w, ctx, C4_SPECS, p, replays=2)
    assert 1 <= grid <= ntiles
    if p == w.F32:
        _check_items(keep, results, C4_SPECS, 1e-5, site_tol=1e-5)
    else:
        _check_items(keep, results, C4_SPECS, 5e-3)
    for k in keep:
        k[1].close()
    ctx.close()


def test_batch_run_refuses_a_gauge_whose_temporal_state_changed(w):
    """A batch captured on plain links must not run on links fixed to the temporal gauge
    since (the captured kernel would load t-links the fixed field no longer needs, and the
    reverse would skip links that are not the identity); a re-upload in the captured state
    is fine."""
    import torch
    ctx = w.Context(0)
    dims = (4, 4, 4, 8)
    U, psi = _inputs(dims, 4200, 1)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    fin = w.pack(ctx, lat, w.ODD, w.F32, psi, 1)
    fout = w.new_field(lat, w.EVEN, w.F32, 1)
    items = (w.WdBatchItem * 1)()
    items[0].gauge, items[0].out_subset, items[0].dagger, items[0].nrhs = g.handle.value, w.EVEN, 0, 1
    items[0].in_, items[0].out = fin.data_ptr(), fout.data_ptr()
    b = ctypes.c_void_p()
    w.wd_batch_create(ctx.handle, 1, items, w.F32, ctypes.byref(b))
    lib = w._raw()
    U2 = ls.gauge_field(dims, 0.5, 4201)
    g.upload(U2)                                   # same (unfixed) state: runs, on the new links
    assert lib.wd_batch_run(b) == w.WD_OK
    torch.cuda.synchronize()
    got = w.unpack(ctx, lat, w.EVEN, w.F32, fout, psi.shape, 1)
    assert orc.rel_l2(got[0], orc.d_eo(U2, psi[0], BC)) < 1e-5
    w.wd_gauge_fix_temporal(g.handle, None)
    fout.fill_(7)
    assert lib.wd_batch_run(b) == w.WD_EINVAL      # state changed: refused, nothing written
    assert b"create the batch again" in lib.wd_last_error()
    torch.cuda.synchronize()
    assert int((fout != 7).sum()) == 0
    w.wd_batch_destroy(b)
    g.close()
    ctx.close()
