"""GPU: temporal gauge fixing. The library's rotation Omega is checked
independently (unitarity; the oracle-side transform of the links gives unit
t-links on all but the last slice), and the dslash that skips the unit links
matches the FP64 oracle applied to the transformed links and, by covariance,
Omega times the oracle on the original links."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS = (4, 6, 4, 8)


def transform(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        out[mu] = Om @ U[mu] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=ax), -1, -2))
    return out


@pytest.fixture(scope="module")
def fixed():
    from paper_0810_5365_amd import wdirac as w
    ctx = w.Context(0)
    U = ls.gauge_field(DIMS, 0.5, 77)
    X, Y, Z, T = DIMS
    out = {}
    for recon in (12, 18):
        g = w.Gauge(ctx, DIMS, BC, recon)
        g.upload(U)
        Om = np.empty((T, Z, Y, X, 3, 3), dtype=np.complex128)
        w.wd_gauge_fix_temporal(g.handle, Om.ctypes.data)
        out[recon] = (g, Om)
    yield w, ctx, U, out
    for g, _ in out.values():
        g.close()
    ctx.close()


def test_rotation_is_su3_and_fixes_time_links(fixed):
    w, ctx, U, out = fixed
    g, Om = out[12]
    eye = np.eye(3)
    assert np.abs(Om @ np.conj(np.swapaxes(Om, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(Om) - 1).max() < 1e-13
    Up = transform(U, Om)
    assert np.abs(Up[3][:-1] - eye).max() < 1e-13          # t = 0 .. T-2
    assert np.abs(Up[3][-1] - eye).max() > 0.1              # the last slice keeps the Polyakov-line product


@pytest.mark.parametrize("recon", [12, 18])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fixed_gauge_dslash_matches_oracle(fixed, recon, prec):
    w, ctx, U, out = fixed
    g, Om = out[recon]
    p = w.PREC_BY_NAME[prec]
    tol = 1e-5 if p == w.F32 else 1e-12
    Up = transform(U, Om)
    X, Y, Z, T = DIMS
    lat = w.lattice(DIMS, BC)
    psi = ls.gaussian_complex((X * Y * Z * T // 2, 4, 3), 5, ls.STREAM_SPINOR)
    for out_sub, in_sub, ref in ((w.EVEN, w.ODD, orc.d_eo), (w.ODD, w.EVEN, orc.d_oe)):
        for dag in (0, 1):
            fin = w.pack(ctx, lat, in_sub, p, psi)
            fo = w.new_field(lat, out_sub, p)
            w.wd_dslash(g.handle, out_sub, dag, p, 1, fin.data_ptr(), fo.data_ptr())
            got = w.unpack(ctx, lat, out_sub, p, fo, psi.shape)
            assert orc.rel_l2(got, ref(Up, psi, BC, bool(dag))) < tol


def test_covariance_of_the_fixed_operator(fixed):
    """M[U'] (Omega psi) = Omega M[U] psi with M from the fixed-gauge GPU kernels."""
    w, ctx, U, out = fixed
    g, Om = out[12]
    lat = w.lattice(DIMS, BC)
    kappa = 0.124
    psi = ls.gaussian_spinor(DIMS, 9)
    rot = lambda f: np.einsum("tzyxab,tzyxsb->tzyxsa", Om, f)
    fin = w.pack(ctx, lat, w.FULL, w.F64, rot(psi))
    fo = w.new_field(lat, w.FULL, w.F64)
    w.wd_apply_M(g.handle, kappa, w.FULL, 0, w.F64, 1, fin.data_ptr(), fo.data_ptr())
    got = w.unpack(ctx, lat, w.FULL, w.F64, fo, psi.shape)
    assert orc.rel_l2(got, rot(orc.apply_m(U, psi, kappa, BC))) < 1e-12


def test_solve_in_fixed_gauge(fixed):
    import torch
    w, ctx, U, out = fixed
    g, Om = out[12]
    lat = w.lattice(DIMS, BC)
    kappa, tol = 0.124, 1e-10
    b = ls.gaussian_spinor(DIMS, 10)
    rot = lambda f: np.einsum("tzyxab,tzyxsb->tzyxsa", Om, f)
    fb = w.pack(ctx, lat, w.FULL, w.F64, rot(b))
    fx = torch.zeros_like(fb)
    prm = w.solver_params(tol=tol, maxiter=1000, sloppy=w.F32)
    info = w.WdSolverInfo()
    w.wd_wilson_solve(g.handle, kappa, ctypes.byref(prm), fb.data_ptr(), fx.data_ptr(), ctypes.byref(info))
    xp = w.unpack(ctx, lat, w.FULL, w.F64, fx, b.shape)
    x = np.einsum("tzyxba,tzyxsb->tzyxsa", np.conj(Om), xp)       # back to the original gauge
    assert orc.rel_residual(lambda v: orc.apply_m(U, v, kappa, BC), x, b) <= 1.05 * tol
