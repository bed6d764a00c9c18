"""GPU: the launch-shape autotuner fills the tuning table, the tuned kernels
still match the FP64 oracle, and the table round-trips through its JSON file."""
import os

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def test_autotune_then_parity_and_cache_roundtrip(tmp_path):
    from paper_0810_5365_amd import wdirac as w
    dims = (8, 8, 8, 16)
    X, Y, Z, T = dims
    ctx = w.Context(0)
    g = w.Gauge(ctx, dims, BC, 12)
    U = ls.gauge_field(dims, 0.5, 17)
    g.upload(U)
    path = str(tmp_path / "tune.json")
    w.wd_autotune_dslash(g.handle, w.F32, 1, path.encode())
    entries = {}
    for dag in (0, 1):
        for xp in (0, 1):
            e = w.tune_get(ctx, w.dslash_key(dims, w.F32, 12, 1, dag, xp))
            assert e is not None and e["block"] in (64, 128, 192, 256) and e["zb"] in (0, 2, 4)
            entries[(dag, xp)] = e
    assert os.path.exists(path) and '"entries"' in open(path).read()
    lat = w.lattice(dims, BC)
    psi = ls.gaussian_complex((X * Y * Z * T // 2, 4, 3), 3, ls.STREAM_SPINOR)
    fin = w.pack(ctx, lat, w.ODD, w.F32, psi)
    fout = w.new_field(lat, w.EVEN, w.F32)
    for dag in (0, 1):
        w.wd_dslash(g.handle, w.EVEN, dag, w.F32, 1, fin.data_ptr(), fout.data_ptr())
        got = w.unpack(ctx, lat, w.EVEN, w.F32, fout, psi.shape)
        assert orc.rel_l2(got, orc.d_eo(U, psi, BC, bool(dag))) < 1e-5
    g.close()
    ctx.close()
    # a fresh context reads the same table back
    ctx2 = w.Context(0)
    w.wd_tune_load(ctx2.handle, path.encode())
    for (dag, xp), e in entries.items():
        assert w.tune_get(ctx2, w.dslash_key(dims, w.F32, 12, 1, dag, xp)) == e
    ctx2.close()


@pytest.mark.parametrize("block,remap,nt,pf,zb", [(64, 0, 0, 0, 0), (128, 1, 1, 0, 2), (192, 1, 0, 1, 5),
                                                   (256, 0, 1, 1, 0), (64, 1, 1, 1, 2)])
def test_every_launch_shape_is_correct(block, remap, nt, pf, zb, monkeypatch):
    """Each shape the tuner may pick gives the oracle's result (set through the
    environment defaults that apply when the table has no entry)."""
    monkeypatch.setenv("WD_DSLASH_BLOCK", str(block))
    monkeypatch.setenv("WD_DSLASH_REMAP", str(remap))
    monkeypatch.setenv("WD_DSLASH_NT", str(nt))
    monkeypatch.setenv("WD_DSLASH_PF", str(pf))
    monkeypatch.setenv("WD_DSLASH_ZB", str(zb))
    from paper_0810_5365_amd import wdirac as w
    dims = (6, 4, 10, 4)
    X, Y, Z, T = dims
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.5, 19)
    for prec, tol in ((w.F32, 1e-5), (w.F64, 1e-12)):
        g = w.Gauge(ctx, dims, BC, 12)
        g.upload(U)
        lat = w.lattice(dims, BC)
        psi = ls.gaussian_complex((2, X * Y * Z * T // 2, 4, 3), 5, ls.STREAM_SPINOR)
        fin = w.pack(ctx, lat, w.ODD, prec, psi, 2)
        fout = w.new_field(lat, w.EVEN, prec, 2)
        w.wd_dslash(g.handle, w.EVEN, 1, prec, 2, fin.data_ptr(), fout.data_ptr())
        got = w.unpack(ctx, lat, w.EVEN, prec, fout, psi.shape, 2)
        ref = orc.d_eo(U, psi, BC, True)
        for r in range(2):
            assert orc.rel_l2(got[r], ref[r]) < tol
        g.close()
    ctx.close()
