"""GPU: the reductions' fallback without a mapped host buffer.

Normally every float64 sum is written by its kernel straight into a mapped host buffer, and
the host spins on that buffer.  With WD_RESULTS_UNMAPPED=1 at context creation the results are
copied behind the kernels instead and the host synchronises the stream.  The kernels and their
fixed-order sums are the same either way, so every result must agree bit for bit: a float64
dot product, and Wilson solves by CG (scalars kept on the device, reliable updates), BiCGstab
and flexible GMRES, each checked as well by the oracle's float64 residual.
"""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS = (8, 8, 8, 16)
KAPPA, TOL = 0.1245, 1e-10


def _solve(w, monkeypatch, unmapped, solver, sloppy):
    import torch
    if unmapped:
        monkeypatch.setenv("WD_RESULTS_UNMAPPED", "1")
    ctx = w.Context(0)
    monkeypatch.delenv("WD_RESULTS_UNMAPPED", raising=False)
    U = ls.gauge_field(DIMS, 0.6, 7101)
    g = w.Gauge(ctx, DIMS, BC, 12)
    g.upload(U)
    lat = w.lattice(DIMS, BC)
    X, Y, Z, T = DIMS
    b = ls.gaussian_complex((T, Z, Y, X, 4, 3), 7102, ls.STREAM_SPINOR)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    fx = torch.zeros_like(fb)
    res = (ctypes.c_double * 2)()
    w.wd_dot(ctx.handle, ctypes.byref(lat), w.FULL, w.F64, 1, fb.data_ptr(), fb.data_ptr(), res)
    prm = w.solver_params(tol=TOL, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy])
    info = w.WdSolverInfo()
    if solver == "cg":
        w.wd_wilson_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    elif solver == "bicgstab":
        w.wd_bicgstab_solve(g.handle, KAPPA, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    else:
        w.wd_fgmres_solve(g.handle, KAPPA, ctypes.byref(prm), 16, 0, None, None, w.F32, fb.data_ptr(),
                          fx.data_ptr(), ctypes.byref(info))
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    out = (res[0], res[1], x, info.as_dict(), orc.rel_residual(lambda v: orc.apply_m(U, v, KAPPA, BC), x, b))
    g.close()
    ctx.close()
    return out


@pytest.mark.parametrize("solver,sloppy", [("cg", "f32"), ("cg", "bf16"), ("bicgstab", "f16"), ("fgmres", "f32")])
def test_unmapped_results_match_the_mapped_path(monkeypatch, solver, sloppy):
    from paper_0810_5365_amd import wdirac as w
    m = _solve(w, monkeypatch, False, solver, sloppy)
    u = _solve(w, monkeypatch, True, solver, sloppy)
    assert m[0] == u[0] and m[1] == u[1]
    assert np.array_equal(m[2], u[2])
    for k in ("iters", "reliable_updates", "operator_applies", "status", "true_resid", "true_resid_M"):
        assert m[3][k] == u[3][k], (k, m[3][k], u[3][k])
    assert m[3]["status"] == w.WD_OK and m[4] <= 1.05 * TOL, (m[3], m[4])
