"""GPU: the closing step of the even-odd solvers (x_o = b_o + kappa D_oe x_e, then the float64
full-system residual) on each of its routes.  D_oe x_e is reused from the last float64 Schur
residual when that was taken at the returned x_e (a converged solve, an iteration cap, a
non-zero guess with no iterations); with a zero guess and no iterations it is a fresh hop.
Every route must rebuild the oracle's x_o and report the oracle's residuals (paper, Section 4:
the even-odd preconditioned system)."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS, KAPPA, TOL = (8, 8, 8, 16), 0.1245, 1e-10


@pytest.fixture(scope="module")
def env():
    from paper_0810_5365_amd import wdirac as w
    ctx = w.Context(0)
    U = ls.gauge_field(DIMS, 0.6, 3021)
    g = w.Gauge(ctx, DIMS, BC, 12)
    g.upload(U)
    yield w, ctx, g, U
    g.close()
    ctx.close()


def _solve(w, g, solver, maxiter, fb, fx):
    prm = w.solver_params(tol=TOL, maxiter=maxiter, sloppy=w.F32)
    info = w.WdSolverInfo()
    ok = (w.WD_OK, w.WD_ENOCONV)
    if solver == "wilson":
        w.wd_wilson_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info), ok=ok)
    elif solver == "bicgstab":
        w.wd_bicgstab_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info), ok=ok)
    else:
        w.wd_fgmres_solve(g.handle, KAPPA, ctypes.byref(prm), 16, 0, None, None, w.F32, fb.data_ptr(), fx.data_ptr(),
                          ctypes.byref(info), ok=ok)
    return info


@pytest.mark.parametrize("solver", ["wilson", "bicgstab", "fgmres"])
@pytest.mark.parametrize("route", ["converged", "capped", "warm_no_iter", "zero_no_iter"])
def test_closing_step_routes(env, solver, route):
    w, ctx, g, U = env
    X, Y, Z, T = DIMS
    lat = w.lattice(DIMS, BC)
    b = ls.gaussian_complex((T, Z, Y, X, 4, 3), 61, ls.STREAM_SPINOR)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    x0 = np.zeros_like(b) if route != "warm_no_iter" else ls.gaussian_complex(b.shape, 62, ls.STREAM_SPINOR)
    fx = w.pack(ctx, lat, w.FULL, w.F64, x0)
    maxiter = {"converged": 2000, "capped": 3, "warm_no_iter": 0, "zero_no_iter": 0}[route]
    if solver == "fgmres" and route == "capped":
        maxiter = 8   # one short cycle: a float64 refinement, short of the tolerance
    info = _solve(w, g, solver, maxiter, fb, fx)
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    x_e = orc.eo_split(x, DIMS, 0)
    # x_o as the oracle builds it from the returned x_e
    ref = orc.schur_reconstruct(U, x_e, b, KAPPA, BC)
    assert orc.rel_l2(orc.eo_split(x, DIMS, 1), orc.eo_split(ref, DIMS, 1)) < 1e-13, info.as_dict()
    # the reported residuals against the oracle's float64 ones
    nb = np.sqrt(orc.norm2(b))
    schur = np.sqrt(orc.norm2(orc.schur_source(U, b, KAPPA, BC) - orc.mhat(U, x_e, KAPPA, BC))) / nb
    full = orc.rel_residual(lambda v: orc.apply_m(U, v, KAPPA, BC), x, b)
    assert abs(info.true_resid_M - full) <= 1e-3 * TOL + 1e-6 * full, (full, info.as_dict())
    if solver != "fgmres":   # FGMRES reports the full-system residual in both fields
        assert abs(info.true_resid - schur) <= 1e-3 * TOL + 1e-6 * schur, (schur, info.as_dict())
    if route == "converged":
        assert info.status == w.WD_OK and full <= 1.05 * TOL
    else:
        assert full > TOL
    # hopping-term applications: bhat (1); the Wilson CG's c = Mhat^dag bhat (2, always formed);
    # with no iteration, the residual of a non-zero guess (Wilson CG: Mhat x_e in float64 and
    # Mhat^dag of it, 4; the other two: Mhat x_e, 2), and the closing hop pair (2) unless x_o
    # reused D_oe x_e
    no_iter = {("wilson", "zero_no_iter"): 1 + 2 + 2, ("wilson", "warm_no_iter"): 1 + 2 + 4,
               ("bicgstab", "zero_no_iter"): 1 + 2, ("bicgstab", "warm_no_iter"): 1 + 2,
               ("fgmres", "zero_no_iter"): 1 + 2, ("fgmres", "warm_no_iter"): 1 + 2}
    if (solver, route) in no_iter:
        assert info.hops == no_iter[(solver, route)], info.as_dict()
    else:   # CG: four per iteration; BiCGstab and FGMRES: two per Mhat
        assert info.hops >= (4 if solver == "wilson" else 2) * info.iters + 1, info.as_dict()
