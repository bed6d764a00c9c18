"""GPU: BiCGstab on the even-odd system reaches the requested full-system
residual, recomputed in FP64 by the oracle on the returned x."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.mark.parametrize("sloppy", ["f64", "f32", "f16", "bf16"])
def test_bicgstab_wilson_system(sloppy):
    import torch
    from paper_0810_5365_amd import wdirac as w
    dims, kappa, tol = (8, 8, 8, 16), 0.1245, 1e-10
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.6, 3001)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    b = ls.gaussian_spinor(dims, 41)
    fb = w.pack(ctx, lat, w.FULL, w.F64, b)
    fx = torch.zeros_like(fb)
    prm = w.solver_params(tol=tol, maxiter=2000, sloppy=w.PREC_BY_NAME[sloppy], delta=0.1)
    info = w.WdSolverInfo()
    w.wd_bicgstab_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    x = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    res = orc.rel_residual(lambda v: orc.apply_m(U, v, kappa, BC), x, b)
    assert info.status == w.WD_OK
    assert res <= 1.05 * tol, (res, info.as_dict())
    assert abs(res - info.true_resid_M) < 1e-12
    g.close()
    ctx.close()


def test_bicgstab_rejects_bad_params():
    from paper_0810_5365_amd import wdirac as w
    dims = (4, 4, 4, 4)
    ctx = w.Context(0)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(ls.gauge_field(dims, 0.5, 1))
    lat = w.lattice(dims, BC)
    f = w.new_field(lat, w.FULL, w.F64)
    info = w.WdSolverInfo()
    for prm in (w.solver_params(sloppy=7), w.solver_params(tol=-1.0), w.solver_params(delta=1.5)):
        assert w._raw().wd_bicgstab_solve(g.handle, 0.1, ctypes.byref(prm), f.data_ptr(), f.data_ptr(),
                                          ctypes.byref(info)) == w.WD_EINVAL
    g.close()
    ctx.close()
