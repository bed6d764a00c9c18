"""GPU parity: every operator of the HIP library against the FP64 oracle on the
same seeded inputs, through the C ABI.

Bars: FP32 storage <= 1e-5 relative L2 (expected ~1e-7), FP64 <= 1e-12,
16-bit storage <= 5e-3 against the unquantised oracle and within one code
step of the oracle applied to the same quantised inputs; packing is
bit-exact against the oracle's codec emulation.
"""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu

BC = (1, 1, 1, -1)
TOL = {0: 1e-12, 1: 1e-5}   # by precision id: F64, F32


@pytest.fixture(scope="module")
def w():
    from paper_0810_5365_amd import wdirac
    return wdirac


_FIELDS = {}


@pytest.fixture(scope="module")
def ctx(w):
    c = w.Context(0)
    yield c
    # gauge objects must go before their context
    for _, g in _FIELDS.values():
        g.close()
    _FIELDS.clear()
    c.close()


def gauge(w, ctx, dims, eps, seed, recon):
    key = (dims, eps, seed, recon)
    if key not in _FIELDS:
        U = ls.gauge_field(dims, eps, seed)
        g = w.Gauge(ctx, dims, BC, recon)
        g.upload(U)
        _FIELDS[key] = (U, g)
    return _FIELDS[key]


def shape_of(w, dims, subset, nrhs=1):
    X, Y, Z, T = dims
    s = (T, Z, Y, X, 4, 3) if subset == w.FULL else (X * Y * Z * T // 2, 4, 3)
    return s if nrhs == 1 else (nrhs,) + s


def source(w, dims, subset, seed, nrhs=1):
    return ls.gaussian_complex(shape_of(w, dims, subset, nrhs), seed, ls.STREAM_SPINOR)


def run_op(w, ctx, fn, lat, in_subset, out_subset, prec, canon_in, nrhs=1):
    dims = tuple(lat.dims)
    fin = w.pack(ctx, lat, in_subset, prec, canon_in, nrhs)
    fout = w.new_field(lat, out_subset, prec, nrhs)
    fn(fin, fout)
    return w.unpack(ctx, lat, out_subset, prec, fout, shape_of(w, dims, out_subset, nrhs), nrhs)


def ref_dslash(U, psi, subset, dagger, w):
    if subset == w.EVEN:
        return orc.d_eo(U, psi, BC, dagger)
    if subset == w.ODD:
        return orc.d_oe(U, psi, BC, dagger)
    return orc.dhop(U, psi, BC, dagger)


def ref_m(U, psi, kappa, subset, dagger, w):
    if subset == w.FULL:
        return orc.apply_m(U, psi, kappa, BC, dagger)
    return orc.mhat(U, psi, kappa, BC, dagger, parity=0 if subset == w.EVEN else 1)


def in_subset_of(w, out_subset):
    return {w.EVEN: w.ODD, w.ODD: w.EVEN, w.FULL: w.FULL}[out_subset]


# ---------------------------------------------------------------------------
# packing
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("subset", ["full", "even"])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_pack_unpack_matches_codec(w, ctx, subset, prec):
    dims = (4, 6, 2, 10)
    lat = w.lattice(dims, BC)
    sub, p = w.SUBSET_BY_NAME[subset], w.PREC_BY_NAME[prec]
    psi = source(w, dims, sub, 3, nrhs=2)
    psi[0, 5] = 0.0   # an all-zero site
    packed = w.pack(ctx, lat, sub, p, psi, 2)
    back = w.unpack(ctx, lat, sub, p, packed, psi.shape, 2)
    if p == w.F64:
        assert np.array_equal(back, psi)
    elif p == w.F32:
        assert np.array_equal(back, orc.quantize_links_f32(psi))
    else:
        dec, _, _ = orc.quantize_spinor_sites(psi, prec)
        assert np.array_equal(back, dec)


# ---------------------------------------------------------------------------
# dslash, M, M^dagger M in FP32 / FP64
# ---------------------------------------------------------------------------

DIMS = [(8, 8, 8, 16), (4, 6, 2, 10), (2, 2, 2, 2), (6, 4, 12, 2)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("recon", [12, 18])
def test_dslash_all_subsets_and_daggers(w, ctx, dims, prec, recon):
    U, g = gauge(w, ctx, dims, 0.3, 1000 + sum(dims), recon)
    lat = w.lattice(dims, BC)
    p = w.PREC_BY_NAME[prec]
    for out_subset in (w.EVEN, w.ODD, w.FULL):
        for dagger in (0, 1):
            psi = source(w, dims, in_subset_of(w, out_subset), 7 + dagger)
            got = run_op(w, ctx, lambda a, b: w.wd_dslash(g.handle, out_subset, dagger, p, 1, a.data_ptr(), b.data_ptr()),
                         lat, in_subset_of(w, out_subset), out_subset, p, psi)
            err = orc.rel_l2(got, ref_dslash(U, psi, out_subset, dagger, w))
            assert err < TOL[p], (out_subset, dagger, err)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("subset", ["full", "even", "odd"])
def test_apply_m_and_normal_operator(w, ctx, prec, subset):
    dims, kappa = (8, 8, 8, 16), 0.12
    U, g = gauge(w, ctx, dims, 0.3, 1001, 12)
    lat = w.lattice(dims, BC)
    p, sub = w.PREC_BY_NAME[prec], w.SUBSET_BY_NAME[subset]
    psi = source(w, dims, sub, 11)
    for dagger in (0, 1):
        got = run_op(w, ctx, lambda a, b: w.wd_apply_M(g.handle, kappa, sub, dagger, p, 1, a.data_ptr(), b.data_ptr()),
                     lat, sub, sub, p, psi)
        assert orc.rel_l2(got, ref_m(U, psi, kappa, sub, dagger, w)) < TOL[p]
    got = run_op(w, ctx, lambda a, b: w.wd_apply_MdagM(g.handle, kappa, sub, p, 1, a.data_ptr(), b.data_ptr()),
                 lat, sub, sub, p, psi)
    ref = ref_m(U, ref_m(U, psi, kappa, sub, 0, w), kappa, sub, 1, w)
    assert orc.rel_l2(got, ref) < TOL[p]


def test_dslash_xpay(w, ctx):
    dims = (4, 6, 2, 10)
    U, g = gauge(w, ctx, dims, 0.5, 77, 12)
    lat = w.lattice(dims, BC)
    psi_o = source(w, dims, w.ODD, 1)
    x_e = source(w, dims, w.EVEN, 2)
    fin = w.pack(ctx, lat, w.ODD, w.F32, psi_o)
    fx = w.pack(ctx, lat, w.EVEN, w.F32, x_e)
    fout = w.new_field(lat, w.EVEN, w.F32)
    w.wd_dslash_xpay(g.handle, w.EVEN, 1, w.F32, 1, fin.data_ptr(), fx.data_ptr(), 0.7, -0.3, fout.data_ptr())
    got = w.unpack(ctx, lat, w.EVEN, w.F32, fout, x_e.shape)
    assert orc.rel_l2(got, 0.7 * x_e - 0.3 * orc.d_eo(U, psi_o, BC, True)) < 1e-5
    # in place: out aliases x
    w.wd_dslash_xpay(g.handle, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fx.data_ptr(), 1.0, 2.0, fx.data_ptr())
    got = w.unpack(ctx, lat, w.EVEN, w.F32, fx, x_e.shape)
    assert orc.rel_l2(got, x_e + 2.0 * orc.d_eo(U, psi_o, BC, False)) < 1e-5


@pytest.mark.parametrize("subset", ["full", "even"])
def test_multiple_right_hand_sides(w, ctx, subset):
    dims, nrhs = (4, 6, 2, 10), 3
    U, g = gauge(w, ctx, dims, 0.5, 78, 12)
    lat = w.lattice(dims, BC)
    sub = w.SUBSET_BY_NAME[subset]
    psi = source(w, dims, in_subset_of(w, sub), 5, nrhs)
    got = run_op(w, ctx, lambda a, b: w.wd_dslash(g.handle, sub, 0, w.F32, nrhs, a.data_ptr(), b.data_ptr()),
                 lat, in_subset_of(w, sub), sub, w.F32, psi, nrhs)
    ref = ref_dslash(U, psi, sub, 0, w)
    for r in range(nrhs):
        assert orc.rel_l2(got[r], ref[r]) < 1e-5


# ---------------------------------------------------------------------------
# 16-bit storage
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f16", "bf16"])
@pytest.mark.parametrize("recon", [12, 18])
def test_dslash_16bit_storage(w, ctx, prec, recon):
    dims = (8, 8, 8, 16)
    U, g = gauge(w, ctx, dims, 0.3, 1001, recon)
    lat = w.lattice(dims, BC)
    p = w.PREC_BY_NAME[prec]
    psi = source(w, dims, w.ODD, 21)
    got = run_op(w, ctx, lambda a, b: w.wd_dslash(g.handle, w.EVEN, 0, p, 1, a.data_ptr(), b.data_ptr()),
                 lat, w.ODD, w.EVEN, p, psi)
    # storage error budget against the unquantised FP64 operator
    err = orc.rel_l2(got, orc.d_eo(U, psi, BC))
    assert err < 5e-3, err
    # arithmetic: the oracle on the same quantised inputs, within one code step of the output scale
    Uq = orc.quantize_links(U, prec)
    if recon == 12:
        Uq = orc.reconstruct12(Uq)
    psi_q, _, _ = orc.quantize_spinor_sites(psi, prec)
    ref = orc.d_eo(Uq, psi_q, BC)
    step = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}[prec]
    scale = np.abs(np.stack([ref.real, ref.imag], -1)).reshape(ref.shape[0], -1).max(axis=1)
    diff = np.abs(np.stack([(got - ref).real, (got - ref).imag], -1)).reshape(ref.shape[0], -1).max(axis=1)
    assert np.all(diff <= scale * (step + 1e-5))


# ---------------------------------------------------------------------------
# float64 global sums
# ---------------------------------------------------------------------------

def test_dot_and_norm_are_float64_and_deterministic(w, ctx):
    dims = (8, 8, 8, 16)
    lat = w.lattice(dims, BC)
    a = source(w, dims, w.FULL, 1, 2)
    b = source(w, dims, w.FULL, 2, 2)
    fa = w.pack(ctx, lat, w.FULL, w.F64, a, 2)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b, 2)
    res = (ctypes.c_double * 2)()
    w.wd_dot(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 2, fa.data_ptr(), fb.data_ptr(), res)
    d = complex(res[0], res[1])
    ref = orc.dot(a, b)
    assert abs(d - ref) < 1e-13 * abs(ref) * 100
    res2 = (ctypes.c_double * 2)()
    w.wd_dot(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 2, fa.data_ptr(), fb.data_ptr(), res2)
    assert res[0] == res2[0] and res[1] == res2[1]
    n = (ctypes.c_double * 1)()
    w.wd_norm2(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 2, fa.data_ptr(), n)
    assert abs(n[0] - orc.norm2(a)) < 1e-13 * orc.norm2(a)


# ---------------------------------------------------------------------------
# solvers: the oracle recomputes the residual in FP64 on the returned x
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sloppy", ["f64", "f32", "f16", "bf16"])
def test_cg_even_odd_normal_equations(w, ctx, sloppy):
    dims, kappa, tol = (8, 8, 8, 16), 0.1245, 1e-10
    U, g = gauge(w, ctx, dims, 0.6, 3001, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 31)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=tol, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    x = w.unpack(ctx, lat, w.EVEN, w.F64, fx, c.shape)
    res = orc.rel_residual(lambda v: orc.mhat_dag_mhat(U, v, kappa, BC), x, c)
    assert info.status == w.WD_OK
    assert res <= 1.05 * tol, (res, info.as_dict())
    assert abs(res - info.true_resid) <= 1e-3 * tol + 1e-2 * res
    # every counted application (an iteration's Mhat^dag Mhat, a residual's Mhat then Mhat^dag)
    # is four hops on one parity
    assert info.hops == 4 * info.operator_applies, info.as_dict()


@pytest.mark.parametrize("sloppy", ["f64", "f32", "bf16"])
def test_cg_full_lattice_normal_equations(w, ctx, sloppy):
    """CG on M^dag M x = c over both parities (the residual update fused into both launches
    of M^dag), checked by the oracle's float64 residual."""
    dims, kappa, tol = (8, 8, 8, 8), 0.12, 1e-10
    U, g = gauge(w, ctx, dims, 0.6, 3005, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.FULL, 37)
    fb = w.pack(ctx, lat, w.FULL, w.F64, c)
    fx = w.pack(ctx, lat, w.FULL, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=tol, maxiter=3000, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    w.wd_cg_solve(g.handle, kappa, w.FULL, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, c.shape)
    res = orc.rel_residual(lambda v: orc.apply_mdagm(U, v, kappa, BC), x, c)
    assert info.status == w.WD_OK
    assert res <= 1.05 * tol, (res, info.as_dict())
    assert abs(res - info.true_resid) <= 1e-3 * tol + 1e-2 * res
    # M^dag M on the full lattice is two full hops, each one hop per parity
    assert info.hops == 4 * info.operator_applies, info.as_dict()


@pytest.mark.parametrize("sloppy", ["f32", "bf16"])
def test_wilson_solve_full_system(w, ctx, sloppy):
    dims, kappa, tol = (8, 8, 8, 16), 0.1245, 1e-10
    U, g = gauge(w, ctx, dims, 0.6, 3001, 12)
    lat = w.lattice(dims, BC)
    b = source(w, dims, w.FULL, 41)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    fx = w.pack(ctx, lat, w.FULL, w.F64, np.zeros_like(b))
    prm = w.solver_params(tol=tol, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    w.wd_wilson_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    res = orc.rel_residual(lambda v: orc.apply_m(U, v, kappa, BC), x, b)
    assert info.status == w.WD_OK
    assert res <= 1.05 * tol, (res, info.as_dict())


@pytest.mark.parametrize("sloppy,delta", [("f32", 0.1), ("f32", 1e-4), ("f32", -1.0), ("f16", -1.0), ("bf16", 0.1), ("bf16", -1.0)])
def test_cg_reliable_update_thresholds(w, ctx, sloppy, delta):
    """Explicit and default (delta < 0) reliable-update thresholds reach the FP64-checked
    tolerance; the number of updates falls as delta does."""
    dims, kappa, tol = (8, 8, 8, 16), 0.1245, 1e-10
    U, g = gauge(w, ctx, dims, 0.6, 3002, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 32)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    runs = {}
    for d in (delta, 0.3):
        fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
        prm = w.solver_params(tol=tol, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy], delta=d)
        info = w.WdSolverInfo()
        w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
        x = w.unpack(ctx, lat, w.EVEN, w.F64, fx, c.shape)
        res = orc.rel_residual(lambda v: orc.mhat_dag_mhat(U, v, kappa, BC), x, c)
        assert info.status == w.WD_OK and res <= 1.05 * tol, (d, res, info.as_dict())
        runs[d] = info.reliable_updates
    assert runs[delta] <= runs[0.3]


def test_cg_rejects_bad_delta(w, ctx):
    dims = (4, 4, 4, 4)
    U, g = gauge(w, ctx, dims, 0.5, 3003, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 33)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
    lib = w._raw()
    for d in (1.0, 2.5, float("nan")):
        prm = w.solver_params(tol=1e-8, maxiter=100, sloppy=w.F32, delta=d)
        info = w.WdSolverInfo()
        assert lib.wd_cg_solve(g.handle, 0.12, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(),
                               ctypes.byref(info)) == w.WD_EINVAL


def test_cg_pure_sloppy_stalls_at_single_precision(w, ctx):
    """Without reliable updates the FP32 recurrences stop where the iterated residual
    meets the target; the FP64-checked residual then sits far above it."""
    dims, kappa, tol = (8, 8, 8, 16), 0.1245, 1e-12
    U, g = gauge(w, ctx, dims, 0.6, 3004, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 34)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=tol, maxiter=3000, sloppy=w.F32, pure_sloppy=True)
    info = w.WdSolverInfo()
    w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info),
                  ok=(w.WD_OK, w.WD_ENOCONV))
    x = w.unpack(ctx, lat, w.EVEN, w.F64, fx, c.shape)
    res = orc.rel_residual(lambda v: orc.mhat_dag_mhat(U, v, kappa, BC), x, c)
    assert info.reliable_updates == 0 and info.status == w.WD_ENOCONV
    assert 1e-9 < res < 1e-4 and abs(res - info.true_resid) <= 1e-2 * res


def test_cg_maxiter_reports_noconv(w, ctx):
    dims, kappa = (4, 6, 2, 10), 0.124
    U, g = gauge(w, ctx, dims, 0.5, 77, 12)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 3)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=1e-12, maxiter=2, sloppy=w.F32)
    info = w.WdSolverInfo()
    s = w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info),
                      ok=(w.WD_OK, w.WD_ENOCONV))
    assert s == w.WD_ENOCONV and info.status == w.WD_ENOCONV
    assert info.iters == 2 and 0 < info.true_resid < 1


def _dense_mdagm_spectrum(U, dims, kappa):
    """Eigenvalues of the oracle's Mhat^dag Mhat as a dense matrix (unit vectors in)."""
    n = dims[0] * dims[1] * dims[2] * dims[3] // 2 * 12
    A = np.empty((n, n), complex)
    for i in range(n):
        e = np.zeros(n, complex)
        e[i] = 1.0
        A[:, i] = orc.mhat_dag_mhat(U, e.reshape(-1, 4, 3), kappa, BC).reshape(-1)
    return np.linalg.eigvalsh(A)


@pytest.mark.parametrize("sloppy,solver", [("f64", "cg"), ("f32", "cg"), ("f32", "wilson")])
def test_cg_ritz_values_match_the_spectrum_ends(w, ctx, sloppy, solver):
    """The extreme Ritz values the CG reports (from its step lengths and residual ratios)
    against the ends of the spectrum of the oracle's dense Mhat^dag Mhat on 4^4: inside
    the spectrum, and within 1% of its ends once the solve has converged."""
    dims, kappa = (4, 4, 4, 4), 0.124
    U, g = gauge(w, ctx, dims, 0.3, 3003, 12)
    ev = _dense_mdagm_spectrum(U, dims, kappa)
    lat = w.lattice(dims, BC)
    sub = w.EVEN if solver == "cg" else w.FULL
    c = source(w, dims, sub, 35)
    fb = w.pack(ctx, lat, sub, w.F64, c)
    fx = w.pack(ctx, lat, sub, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=1e-12, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    if solver == "cg":
        w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    else:
        w.wd_wilson_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    assert info.status == w.WD_OK
    # a lattice spectrum is dense at both ends, so the extreme Ritz values approach them
    # slowly (1e-3 after the 40 iterations to 1e-12 here); the float32 iterations perturb
    # the coefficients, which may move them slightly outside
    out = 1e-9 if sloppy == "f64" else 1e-4
    lo, hi = info.lambda_min, info.lambda_max
    assert ev[0] * (1 - out) <= lo <= ev[0] * (1 + 1e-2), (lo, ev[0], info.as_dict())
    assert ev[-1] * (1 - 1e-2) <= hi <= ev[-1] * (1 + out), (hi, ev[-1], info.as_dict())


def test_cg_ritz_values_of_a_short_run_lie_inside(w, ctx):
    """Two iterations: the Ritz values of the 2x2 tridiagonal are inside the spectrum
    (Cauchy interlacing) but not yet at its ends."""
    dims, kappa = (4, 4, 4, 4), 0.124
    U, g = gauge(w, ctx, dims, 0.3, 3003, 12)
    ev = _dense_mdagm_spectrum(U, dims, kappa)
    lat = w.lattice(dims, BC)
    c = source(w, dims, w.EVEN, 36)
    fb = w.pack(ctx, lat, w.EVEN, w.F64, c)
    fx = w.pack(ctx, lat, w.EVEN, w.F64, np.zeros_like(c))
    prm = w.solver_params(tol=1e-12, maxiter=2, sloppy=w.F64)
    info = w.WdSolverInfo()
    w.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info),
                  ok=(w.WD_OK, w.WD_ENOCONV))
    assert info.iters == 2
    assert ev[0] < info.lambda_min < info.lambda_max < ev[-1], (info.as_dict(), ev[0], ev[-1])
    assert info.lambda_min > ev[0] * 1.01


def test_bad_arguments_leave_outputs_untouched(w, ctx):
    dims = (4, 4, 4, 4)
    U, g = gauge(w, ctx, dims, 0.5, 5, 12)
    lat = w.lattice(dims, BC)
    fin = w.pack(ctx, lat, w.ODD, w.F32, source(w, dims, w.ODD, 1))
    fout = w.new_field(lat, w.EVEN, w.F32)
    fout.fill_(7)
    lib = w._raw()
    assert lib.wd_dslash(g.handle, 9, 0, w.F32, 1, fin.data_ptr(), fout.data_ptr()) == w.WD_EINVAL
    assert lib.wd_dslash(g.handle, w.EVEN, 0, 11, 1, fin.data_ptr(), fout.data_ptr()) == w.WD_EINVAL
    assert lib.wd_dslash(g.handle, w.EVEN, 0, w.F32, 0, fin.data_ptr(), fout.data_ptr()) == w.WD_EINVAL
    assert lib.wd_apply_M(g.handle, 0.1, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fin.data_ptr()) == w.WD_EINVAL
    assert int((fout != 7).sum()) == 0
    empty = ctypes.c_void_p()
    assert lib.wd_gauge_create(ctx.handle, ctypes.byref(w.lattice((3, 4, 4, 4))), 12, ctypes.byref(empty)) == w.WD_ESHAPE
    h = ctypes.c_void_p()
    assert lib.wd_gauge_create(ctx.handle, ctypes.byref(lat), 12, ctypes.byref(h)) == w.WD_OK
    # not uploaded yet
    assert lib.wd_dslash(h, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fout.data_ptr()) == w.WD_EINVAL
    assert lib.wd_gauge_destroy(h) == w.WD_OK


# ---------------------------------------------------------------------------
# the benchmark workload at full size (32^3 x 64, FP32, 12-real links)
# ---------------------------------------------------------------------------

def test_full_size_even_odd_dslash_32c64(w, ctx):
    dims = (32, 32, 32, 64)
    U = ls.gauge_field(dims, 0.5, ls.link_seed(2))
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    X, Y, Z, T = dims
    psi_o = ls.gaussian_complex((X * Y * Z * T // 2, 4, 3), ls.source_seed(2), ls.STREAM_SPINOR)
    got = run_op(w, ctx, lambda a, b: w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, a.data_ptr(), b.data_ptr()),
                 lat, w.ODD, w.EVEN, w.F32, psi_o)
    ref = orc.d_eo(U, psi_o, BC)
    assert orc.rel_l2(got, ref) < 1e-5
    g.close()
