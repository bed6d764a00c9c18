"""GPU: every solver started from a non-zero initial guess (a random field, and the
converged solution itself) reaches the FP64-checked tolerance; a zero guess takes
the shortcut that skips the first operator application (one application fewer)."""
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
    U = ls.gauge_field(DIMS, 0.6, 3011)
    g = w.Gauge(ctx, DIMS, BC, 12)
    g.upload(U)
    yield w, ctx, g, U
    g.close()
    ctx.close()


def _solve(w, g, name, fb, fx):
    prm = w.solver_params(tol=TOL, maxiter=3000, sloppy=w.F32)
    info = w.WdSolverInfo()
    if name == "cg_even":
        w.wd_cg_solve(g.handle, KAPPA, w.EVEN, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    elif name == "wilson":
        w.wd_wilson_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    elif name == "bicgstab":
        w.wd_bicgstab_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    else:
        w.wd_fgmres_solve(g.handle, KAPPA, ctypes.byref(prm), 16, 0, None, None, w.F32, fb.data_ptr(), fx.data_ptr(),
                          ctypes.byref(info))
    return info


@pytest.mark.parametrize("name", ["cg_even", "wilson", "bicgstab", "fgmres"])
def test_solvers_from_nonzero_guesses(env, name):
    import torch
    w, ctx, g, U = env
    X, Y, Z, T = DIMS
    lat = w.lattice(DIMS, BC)
    sub = w.EVEN if name == "cg_even" else w.FULL
    shape = (X * Y * Z * T // 2, 4, 3) if sub == w.EVEN else (T, Z, Y, X, 4, 3)
    b = ls.gaussian_complex(shape, 81, ls.STREAM_SPINOR)
    if sub == w.EVEN:
        op = lambda v: orc.mhat_dag_mhat(U, v, KAPPA, BC)
    else:
        op = lambda v: orc.apply_m(U, v, KAPPA, BC)
    fb = w.pack(ctx, lat, sub, w.F64, b)
    fx = torch.zeros_like(fb)
    zero = _solve(w, g, name, fb, fx)
    x = w.unpack(ctx, lat, sub, w.F64, fx, shape)
    assert zero.status == w.WD_OK and orc.rel_residual(op, x, b) <= 1.05 * TOL
    # a random guess
    g0 = ls.gaussian_complex(shape, 83, ls.STREAM_SPINOR)
    fx = w.pack(ctx, lat, sub, w.F64, g0)
    rnd = _solve(w, g, name, fb, fx)
    xr = w.unpack(ctx, lat, sub, w.F64, fx, shape)
    assert rnd.status == w.WD_OK and orc.rel_residual(op, xr, b) <= 1.05 * TOL, rnd.as_dict()
    # the solution itself: converged before the first iteration, x returned as given
    fx = w.pack(ctx, lat, sub, w.F64, x)
    done = _solve(w, g, name, fb, fx)
    xd = w.unpack(ctx, lat, sub, w.F64, fx, shape)
    assert done.status == w.WD_OK and done.iters == 0, done.as_dict()
    if name != "fgmres":   # FGMRES uses only the even half of the guess and rebuilds x_o
        assert np.array_equal(xd, x)
    assert orc.rel_residual(op, xd, b) <= 1.05 * TOL
    # applications of the operator: one per iteration (two for BiCGstab) and one per reliable
    # update (the last of which finds convergence); a zero guess needs none for its first
    # residual, any other guess one.  The even-odd solvers' closing step applies none here: each
    # solve ends on a float64 residual taken at the returned x_e, whose D_oe x_e builds x_o
    if name != "fgmres":
        per_it = 2 if name == "bicgstab" else 1
        closing = 0
        assert zero.operator_applies == per_it * zero.iters + zero.reliable_updates + closing, zero.as_dict()
        assert rnd.operator_applies == per_it * rnd.iters + rnd.reliable_updates + closing + 1, rnd.as_dict()
        assert done.operator_applies == 1 + closing, done.as_dict()
