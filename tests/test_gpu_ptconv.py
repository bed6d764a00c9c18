"""GPU: parallel-transport convolution forward and both gradients against the
FP64 oracle, the Wilson operator as a special case of the layer, and the
torch.autograd wrapper's gradients against the oracle's analytic chain."""
import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
DIMS = (4, 6, 2, 10)


@pytest.fixture(scope="module")
def env():
    from paper_0810_5365_amd import wdirac as w
    ctx = w.Context(0)
    U = ls.gauge_field(DIMS, 0.7, 5001)
    g = w.Gauge(ctx, DIMS, BC, 12)
    g.upload(U)
    yield w, ctx, U, g, w.lattice(DIMS, BC)
    g.close()
    ctx.close()


def feat(C, seed, n=None):
    X, Y, Z, T = DIMS
    shape = (C, T, Z, Y, X, 3) if n is None else (n, C, T, Z, Y, X, 3)
    return ls.gaussian_complex(shape, seed)


def as_torch_weights(W):
    import torch
    return torch.from_numpy(np.stack([W.real, W.imag], -1).astype(np.float32)).cuda().contiguous()


@pytest.mark.parametrize("cin,cout", [(4, 8), (8, 8), (8, 4), (2, 3), (1, 1), (3, 2)])
def test_forward_matches_oracle(env, cin, cout):
    w, ctx, U, g, lat = env
    n = 2
    phi = feat(cin, 10 + cin, n)
    W = ls.gaussian_complex((9, cout, cin), 20 + cout)
    fin = w.pack_features(ctx, lat, phi, cin, n)
    out = w.pack_features(ctx, lat, np.zeros((n, cout) + phi.shape[2:], complex), cout, n)
    Wt = as_torch_weights(W)
    w.wd_ptconv_forward(g.handle, cin, cout, w.F32, n, Wt.data_ptr(), fin.data_ptr(), out.data_ptr())
    got = w.unpack_features(ctx, lat, out, (n, cout) + phi.shape[2:], cout, n)
    for s in range(n):
        assert orc.rel_l2(got[s], orc.ptconv_forward(U, phi[s], W, BC)) < 1e-5


@pytest.mark.parametrize("wprec", ["bf16", "f16"])
def test_forward_16bit_weights(env, wprec, monkeypatch):
    """Vector-unit path with 16-bit weights: exact up to float32 against the oracle with the same weights."""
    import torch
    monkeypatch.setenv("WD_PTCONV_MFMA", "0")
    w, ctx, U, g, lat = env
    cin, cout = 4, 8
    phi = feat(cin, 31)
    W = ls.gaussian_complex((9, cout, cin), 32)
    fin = w.pack_features(ctx, lat, phi, cin)
    out = w.pack_features(ctx, lat, np.zeros((cout,) + phi.shape[1:], complex), cout)
    dt = torch.bfloat16 if wprec == "bf16" else torch.float16
    Wq = as_torch_weights(W).to(dt).contiguous()
    w.wd_ptconv_forward(g.handle, cin, cout, w.PREC_BY_NAME[wprec], 1, Wq.data_ptr(), fin.data_ptr(), out.data_ptr())
    got = w.unpack_features(ctx, lat, out, (cout,) + phi.shape[1:], cout)
    Wref = orc.round16(W.real.astype(np.float32), wprec) + 1j * orc.round16(W.imag.astype(np.float32), wprec)
    assert orc.rel_l2(got, orc.ptconv_forward(U, phi, Wref.astype(np.complex128), BC)) < 1e-5


def test_wilson_operator_as_a_layer(env):
    """Spin as channels, W_0 = 1, W_{+mu} = -kappa (1 - gamma_mu), W_{-mu} = -kappa (1 + gamma_mu) gives M."""
    w, ctx, U, g, lat = env
    kappa = 0.1248
    X, Y, Z, T = DIMS
    psi = ls.gaussian_spinor(DIMS, 41)
    gm = [orc.gamma(mu) for mu in range(4)]
    W = np.zeros((9, 4, 4), complex)
    W[0] = np.eye(4)
    for mu in range(4):
        W[1 + mu] = -kappa * (np.eye(4) - gm[mu])
        W[5 + mu] = -kappa * (np.eye(4) + gm[mu])
    from paper_0810_5365_amd import ptconv as pt
    sp = w.pack(ctx, lat, w.FULL, w.F32, psi)
    f = pt.spinor_to_features(ctx, lat, sp)
    out = f.clone()
    Wt = as_torch_weights(W)
    w.wd_ptconv_forward(g.handle, 4, 4, w.F32, 1, Wt.data_ptr(), f.data_ptr(), out.data_ptr())
    sp_out = pt.features_to_spinor(ctx, lat, out)
    got = w.unpack(ctx, lat, w.FULL, w.F32, sp_out, psi.shape)
    assert orc.rel_l2(got, orc.apply_m(U, psi, kappa, BC)) < 1e-5


@pytest.mark.parametrize("cin,cout", [(4, 8), (8, 4), (2, 3)])
def test_backward_matches_oracle(env, cin, cout):
    w, ctx, U, g, lat = env
    n = 2
    phi = feat(cin, 50 + cin, n)
    gout = feat(cout, 60 + cout, n)
    W = ls.gaussian_complex((9, cout, cin), 70)
    import torch
    fin = w.pack_features(ctx, lat, phi, cin, n)
    fgo = w.pack_features(ctx, lat, gout, cout, n)
    gin = torch.empty_like(fin)
    gW = torch.empty((9, cout, cin, 2), dtype=torch.float32, device="cuda")
    Wt = as_torch_weights(W)
    w.wd_ptconv_backward(g.handle, cin, cout, w.F32, n, Wt.data_ptr(), fin.data_ptr(), fgo.data_ptr(),
                         gin.data_ptr(), gW.data_ptr())
    got_in = w.unpack_features(ctx, lat, gin, phi.shape, cin, n)
    for s in range(n):
        assert orc.rel_l2(got_in[s], orc.ptconv_backward_input(U, gout[s], W, BC)) < 1e-5
    ref_W = sum(orc.ptconv_backward_weight(U, phi[s], gout[s], BC) for s in range(n))
    gWc = gW.cpu().numpy().astype(np.float64)
    gWc = gWc[..., 0] + 1j * gWc[..., 1]
    assert orc.rel_l2(gWc, ref_W) < 1e-5


def test_autograd_network_gradients(env):
    """Three-layer network (4 -> 8 -> 8 -> 4) through torch.autograd vs the oracle's chain rule."""
    import torch
    from paper_0810_5365_amd import ptconv as pt
    w, ctx, U, g, lat = env
    gen = torch.Generator().manual_seed(3)
    net = pt.PTNet((4, 8, 8, 4), w.F32, generator=gen)
    phi = feat(4, 81)
    x = w.pack_features(ctx, lat, phi, 4).requires_grad_(True)
    y = net(x, g)
    loss = (y * y).sum()
    loss.backward()
    Ws = []
    for Wp in net.weights:
        a = Wp.detach().cpu().numpy().astype(np.float64)
        Ws.append(a[..., 0] + 1j * a[..., 1])
    acts = [phi]
    for W in Ws:
        acts.append(orc.ptconv_forward(U, acts[-1], W, BC))
    gy = 2 * acts[-1]                        # d(sum |y|^2) in the complex convention
    assert abs(loss.item() - orc.norm2(acts[-1])) < 1e-4 * orc.norm2(acts[-1])
    grads = [None] * len(Ws)
    for k in reversed(range(len(Ws))):
        grads[k] = orc.ptconv_backward_weight(U, acts[k], gy, BC)
        gy = orc.ptconv_backward_input(U, gy, Ws[k], BC)
    for Wp, ref in zip(net.weights, grads):
        a = Wp.grad.cpu().numpy().astype(np.float64)
        assert orc.rel_l2(a[..., 0] + 1j * a[..., 1], ref) < 1e-4
    gx = w.unpack_features(ctx, lat, x.grad, phi.shape, 4)
    assert orc.rel_l2(gx, gy) < 1e-4


def test_forward_gauge_covariance_on_gpu(env):
    """N[U^Omega](Omega phi) = Omega N[U] phi for the GPU layer."""
    w, ctx, U, g, lat = env
    Om = ls.gauge_transform(DIMS, 91)
    UO = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        UO[mu] = Om @ U[mu] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=ax), -1, -2))
    gO = w.Gauge(ctx, DIMS, BC, 12)
    gO.upload(UO)
    cin, cout = 2, 3
    phi = feat(cin, 92)
    W = ls.gaussian_complex((9, cout, cin), 93)
    Wt = as_torch_weights(W)
    rot = lambda f: np.einsum("tzyxab,ctzyxb->ctzyxa", Om, f)
    res = []
    for gg, ph in ((g, phi), (gO, rot(phi))):
        fin = w.pack_features(ctx, lat, ph, cin)
        out = w.pack_features(ctx, lat, np.zeros((cout,) + phi.shape[1:], complex), cout)
        w.wd_ptconv_forward(gg.handle, cin, cout, w.F32, 1, Wt.data_ptr(), fin.data_ptr(), out.data_ptr())
        res.append(w.unpack_features(ctx, lat, out, (cout,) + phi.shape[1:], cout))
    assert orc.rel_l2(res[1], rot(res[0])) < 1e-5
    gO.close()


@pytest.mark.parametrize("cin,cout", [(4, 8), (8, 8), (8, 4), (4, 4)])
def test_forward_matrix_core_path(env, cin, cout, monkeypatch):
    """bf16 weights on the MFMA path: the transported inputs are rounded to bf16
    (relative 2^-9 each), so the layer output is within ~2e-3 of the oracle with the
    same weights; bound 1e-2.  Two samples, ragged site count per workgroup."""
    import torch
    monkeypatch.setenv("WD_PTCONV_MFMA", "1")
    w, ctx, U, g, lat = env
    n = 2
    phi = feat(cin, 100 + cin, n)
    W = ls.gaussian_complex((9, cout, cin), 101 + cout)
    Wq = as_torch_weights(W).to(torch.bfloat16).contiguous()
    Wref = orc.round16(W.real.astype(np.float32), "bf16") + 1j * orc.round16(W.imag.astype(np.float32), "bf16")
    fin = w.pack_features(ctx, lat, phi, cin, n)
    out = w.pack_features(ctx, lat, np.zeros((n, cout) + phi.shape[2:], complex), cout, n)
    w.wd_ptconv_forward(g.handle, cin, cout, w.BF16, n, Wq.data_ptr(), fin.data_ptr(), out.data_ptr())
    got = w.unpack_features(ctx, lat, out, (n, cout) + phi.shape[2:], cout, n)
    for s in range(n):
        err = orc.rel_l2(got[s], orc.ptconv_forward(U, phi[s], Wref.astype(np.complex128), BC))
        assert err < 1e-2, err
        assert err > 1e-6          # it did run in bf16


@pytest.mark.parametrize("cin,cout", [(4, 8), (8, 4)])
def test_matrix_core_wave_orders_agree(cin, cout, monkeypatch):
    """The matrix-core layer in the natural and the z-blocked wave order (depths 2 and 4 on a
    16 x 8 x 8 x 8 lattice, where X Y / 2 = 64) gives bit-identical outputs, and matches the
    oracle to the bf16 bound."""
    import torch
    from paper_0810_5365_amd import wdirac as w
    monkeypatch.setenv("WD_PTCONV_MFMA", "1")
    dims = (16, 8, 8, 8)
    X, Y, Z, T = dims
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.7, 5003)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    phi = ls.gaussian_complex((1, cin, T, Z, Y, X, 3), 107)
    W = ls.gaussian_complex((9, cout, cin), 109)
    Wq = as_torch_weights(W).to(torch.bfloat16).contiguous()
    fin = w.pack_features(ctx, lat, phi, cin, 1)
    outs = []
    for zb in ("0", "2", "4"):
        monkeypatch.setenv("WD_PTCONV_ZB", zb)
        out = w.pack_features(ctx, lat, np.zeros((1, cout, T, Z, Y, X, 3), complex), cout, 1)
        w.wd_ptconv_forward(g.handle, cin, cout, w.BF16, 1, Wq.data_ptr(), fin.data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        outs.append(out.clone())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    Wref = orc.round16(W.real.astype(np.float32), "bf16") + 1j * orc.round16(W.imag.astype(np.float32), "bf16")
    got = w.unpack_features(ctx, lat, outs[2], (1, cout, T, Z, Y, X, 3), cout, 1)
    assert orc.rel_l2(got[0], orc.ptconv_forward(U, phi[0], Wref.astype(np.complex128), BC)) < 1e-2
    g.close()
    ctx.close()
