"""GPU: the 16-rhs dslash with the colour multiply on the matrix cores (16-bit storage,
12-real links) against the FP64 oracle and against the per-rhs path, for both
output parities, the dagger, the fused a x + b D in (through Mhat), rhs counts 16
and 32, and a lattice whose last workgroup has waves past the end."""
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


def _hop(w, g, lat, prec, nrhs, psi, out_even, dagger):
    ctx = g.ctx
    fin = w.pack(ctx, lat, w.ODD if out_even else w.EVEN, prec, psi, nrhs)
    fout = w.new_field(lat, w.EVEN if out_even else w.ODD, prec, nrhs)
    w.wd_dslash(g.handle, w.EVEN if out_even else w.ODD, dagger, prec, nrhs, fin.data_ptr(), fout.data_ptr())
    return w.unpack(ctx, lat, w.EVEN if out_even else w.ODD, prec, fout, psi.shape, nrhs)


def _check(got, U, psi, prec_name, out_even, dagger):
    """Storage budget against the unquantised operator, and the oracle on the same
    quantised inputs within one output code step plus the fp16 rounding of the
    matrix-core operands (2^-7 of the output scale)."""
    ref = orc.d_eo(U, psi, BC, dagger) if out_even else orc.d_oe(U, psi, BC, dagger)
    Uq = orc.reconstruct12(orc.quantize_links(U, prec_name))
    step = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[prec_name]
    for r in range(psi.shape[0]):
        assert orc.rel_l2(got[r], ref[r]) < 5e-3
        pq, _, _ = orc.quantize_spinor_sites(psi[r], prec_name)
        refq = orc.d_eo(Uq, pq, BC, dagger) if out_even else orc.d_oe(Uq, pq, BC, dagger)
        scale = np.abs(np.stack([refq.real, refq.imag], -1)).reshape(refq.shape[0], -1).max(axis=1)
        diff = np.abs(np.stack([(got[r] - refq).real, (got[r] - refq).imag], -1)).reshape(refq.shape[0], -1).max(axis=1)
        assert np.all(diff <= scale * (step + 2.0 ** -7)), float((diff / np.maximum(scale, 1e-300)).max())


@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("dims,nrhs,out_even,dagger", [((8, 8, 8, 16), 16, True, 0), ((8, 8, 8, 16), 16, False, 1),
                                                        ((6, 6, 2, 2), 32, True, 1), ((4, 6, 2, 10), 16, False, 0)])
def test_mfma_multi_rhs_dslash(w, monkeypatch, prec, dims, nrhs, out_even, dagger):
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.5, 41)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    p = w.PREC_BY_NAME[prec]
    psi = half_source(dims, 43, nrhs)
    monkeypatch.setenv("WD_DSLASH_MFMA", "1")
    got = _hop(w, g, lat, p, nrhs, psi, out_even, dagger)
    _check(got, U, psi, prec, out_even, dagger)
    # the per-rhs path on the same inputs: both quantise the same way, the products differ
    # only by the fp16 operands
    monkeypatch.setenv("WD_DSLASH_MFMA", "0")
    per_rhs = _hop(w, g, lat, p, nrhs, psi, out_even, dagger)
    for r in range(nrhs):
        assert orc.rel_l2(got[r], per_rhs[r]) < 3e-3
    g.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_mfma_multi_rhs_mhat_and_normal_operator(w, monkeypatch, prec):
    """Mhat (two hops, the second with the fused update) and Mhat^dag Mhat (daggers too),
    16 rhs through the matrix-core path."""
    monkeypatch.setenv("WD_DSLASH_MFMA", "1")
    dims, nrhs, kappa = (8, 8, 8, 16), 16, 0.124
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.5, 47)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    p = w.PREC_BY_NAME[prec]
    psi = half_source(dims, 49, nrhs)
    fin = w.pack(ctx, lat, w.EVEN, p, psi, nrhs)
    for name, fn, ref in (("mhat", w.wd_apply_M, lambda v: orc.mhat(U, v, kappa, BC)),
                          ("mdagm", None, lambda v: orc.mhat_dag_mhat(U, v, kappa, BC))):
        fout = w.new_field(lat, w.EVEN, p, nrhs)
        if name == "mhat":
            w.wd_apply_M(g.handle, kappa, w.EVEN, 0, p, nrhs, fin.data_ptr(), fout.data_ptr())
        else:
            w.wd_apply_MdagM(g.handle, kappa, w.EVEN, p, nrhs, fin.data_ptr(), fout.data_ptr())
        got = w.unpack(ctx, lat, w.EVEN, p, fout, psi.shape, nrhs)
        for r in range(nrhs):
            assert orc.rel_l2(got[r], ref(psi[r])) < 1e-2, (name, r)
    g.close()
    ctx.close()


def test_mfma_path_is_a_tuning_candidate(w, monkeypatch):
    """The autotuner times the matrix-core path for 16-bit multi-rhs calls and records
    its choice; a 16-bit single-rhs call and an FP32 call never select it."""
    monkeypatch.delenv("WD_DSLASH_MFMA", raising=False)
    dims = (8, 8, 8, 16)
    ctx = w.Context(0)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(ls.gauge_field(dims, 0.5, 51))
    w.wd_autotune_dslash(g.handle, w.BF16, 16, None)
    w.wd_autotune_dslash(g.handle, w.BF16, 1, None)
    w.wd_autotune_dslash(g.handle, w.F32, 16, None)
    e16 = w.tune_get(ctx, w.dslash_key(dims, w.BF16, 12, 16, 0, 0))
    e1 = w.tune_get(ctx, w.dslash_key(dims, w.BF16, 12, 1, 0, 0))
    f32 = w.tune_get(ctx, w.dslash_key(dims, w.F32, 12, 16, 0, 0))
    assert e16 is not None and e16["mfma"] in (0, 1)
    assert e1["mfma"] == 0 and f32["mfma"] == 0
    g.close()
    ctx.close()
