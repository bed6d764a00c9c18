"""GPU: the solvers' failure and edge paths, forced from the host with ordinary inputs.

* A source holding NaN or Inf: every solver returns WD_ENAN, fills info (status,
  a non-finite residual) and leaves x as it was; wd_last_error says why.
* An initial guess that already solves the system: WD_OK after no iteration.
* A system the first half-step of BiCGstab solves exactly (free field, periodic
  boundaries, a constant source: an eigenvector of Mhat), where omega = <t, s> / <t, t>
  meets t = s = 0: WD_OK with the oracle's float64 residual below tol, not a breakdown.
"""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS = (4, 4, 4, 8)
KAPPA = 0.124


@pytest.fixture(scope="module")
def env():
    from paper_0810_5365_amd import wdirac as w
    ctx = w.Context(0)
    U = ls.gauge_field(DIMS, 0.5, 7001)
    g = w.Gauge(ctx, DIMS, BC, 12)
    g.upload(U)
    yield w, ctx, U, g
    g.close()
    ctx.close()


def _full_source(seed):
    X, Y, Z, T = DIMS
    return ls.gaussian_complex((T, Z, Y, X, 4, 3), seed, ls.STREAM_SPINOR)


def _call(w, g, solver, fb, fx, prm, info, kappa=KAPPA):
    lib = w._raw()
    if solver == "cg_even":
        return lib.wd_cg_solve(g.handle, kappa, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(),
                               ctypes.byref(info))
    if solver == "wilson":
        return lib.wd_wilson_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    if solver == "bicgstab":
        return lib.wd_bicgstab_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(),
                                     ctypes.byref(info))
    return lib.wd_fgmres_solve(g.handle, kappa, ctypes.byref(prm), 16, 0, None, None, w.F32, fb.data_ptr(),
                               fx.data_ptr(), ctypes.byref(info))


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
@pytest.mark.parametrize("solver", ["cg_even", "wilson", "bicgstab", "fgmres"])
@pytest.mark.parametrize("sloppy", ["f32", "bf16"])
def test_non_finite_source_returns_enan(env, solver, sloppy, bad):
    import torch
    w, ctx, U, g = env
    lat = w.lattice(DIMS, BC)
    b = _full_source(11)
    b[1, 2, 3, 0, 2, 1] = complex(bad, 0.0)
    sub = w.EVEN if solver == "cg_even" else w.FULL
    if sub == w.EVEN:
        b = orc.eo_split(b, DIMS, 0)
    fb = w.pack(ctx, lat, sub, w.F64, b)
    x0 = _full_source(12) if sub == w.FULL else orc.eo_split(_full_source(12), DIMS, 0)
    fx = w.pack(ctx, lat, sub, w.F64, x0)
    before = fx.clone()
    prm = w.solver_params(tol=1e-10, maxiter=100, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    s = _call(w, g, solver, fb, fx, prm, info)
    torch.cuda.synchronize()
    assert s == w.WD_ENAN and info.status == w.WD_ENAN, (s, info.as_dict())
    assert not np.isfinite(info.true_resid) and info.iters == 0
    assert b"NaN or Inf" in w._raw().wd_last_error()
    assert torch.equal(fx, before)


@pytest.mark.parametrize("solver", ["cg_even", "wilson", "bicgstab", "fgmres"])
def test_already_solved_system_is_ok_without_iterating(env, solver):
    """Solve once, then again from the converged x: no iteration, WD_OK, and the oracle's
    residual of the returned x still meets tol."""
    w, ctx, U, g = env
    lat = w.lattice(DIMS, BC)
    b = _full_source(21)
    sub = w.EVEN if solver == "cg_even" else w.FULL
    if sub == w.EVEN:
        b = orc.eo_split(b, DIMS, 0)
    fb = w.pack(ctx, lat, sub, w.F64, b)
    fx = w.pack(ctx, lat, sub, w.F64, np.zeros_like(b))
    prm = w.solver_params(tol=1e-10, maxiter=500, sloppy=w.F32)
    info = w.WdSolverInfo()
    assert _call(w, g, solver, fb, fx, prm, info) == w.WD_OK
    info2 = w.WdSolverInfo()
    assert _call(w, g, solver, fb, fx, prm, info2) == w.WD_OK, info2.as_dict()
    assert info2.iters == 0 and info2.status == w.WD_OK
    x = w.unpack(ctx, lat, sub, w.F64, fx, b.shape)
    if sub == w.EVEN:
        res = orc.rel_residual(lambda v: orc.mhat_dag_mhat(U, v, KAPPA, BC), x, b)
    else:
        res = orc.rel_residual(lambda v: orc.apply_m(U, v, KAPPA, BC), x, b)
    assert res <= 1.05e-10


@pytest.mark.parametrize("sloppy", ["f64", "f32"])
def test_bicgstab_eigenvector_source_converges_in_one_step(env, sloppy):
    """U = 1 with periodic boundaries and a constant source: D_hop psi = 8 psi, so the Schur
    source and every Krylov vector are multiples of one vector, Mhat = (1 - 64 kappa^2) on
    it, and s = r - alpha v vanishes (to rounding) in the first iteration; t = Mhat s then
    vanishes too, which must read as convergence, not as an omega = 0 breakdown."""
    import torch
    w, ctx, _, _ = env
    bc = (1, 1, 1, 1)
    kappa = 1.0 / 16
    U1 = ls.gauge_field(DIMS, 0.0, 1)
    g1 = w.Gauge(ctx, DIMS, bc, 12)
    g1.upload(U1)
    lat = w.lattice(DIMS, bc)
    X, Y, Z, T = DIMS
    b = np.zeros((T, Z, Y, X, 4, 3), complex)
    b[...] = 1.0
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    fx = torch.zeros_like(fb)
    prm = w.solver_params(tol=1e-10, maxiter=20, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    s = w._raw().wd_bicgstab_solve(g1.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(),
                                   ctypes.byref(info))
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    res = orc.rel_residual(lambda v: orc.apply_m(U1, v, kappa, bc), x, b)
    g1.close()
    assert s == w.WD_OK and info.status == w.WD_OK, (s, info.as_dict())
    assert res <= 1.05e-10 and info.iters <= 2, (res, info.as_dict())
    # the exact solution: (1 - 8 kappa) x = b on every site
    assert np.abs(x - b / (1 - 8 * kappa)).max() < 1e-9
