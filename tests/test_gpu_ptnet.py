"""GPU: the learned solve's preconditioner applied on its own (wd_ptnet_apply_even:
the even sites of N (v_e, 0) for a 4 -> 8 -> 8 -> 4 network) against the FP64
oracle's network with the same weights.

Bars.  float32 weights (vector units, float32 features): 1e-5.  bf16 weights
(matrix cores): every layer rounds its transported inputs to bf16 (relative
2^-9 each) and the default path also stores the two hidden feature tensors as
bf16; a rounding error of u = 2^-9 at each of five stages stays well below
1e-2 in the relative L2 norm of the output; the bound is 2e-2.  The bf16 path
must differ from the float32-feature path (it did round), and the float32-feature
path with the parity skip must equal the one without it bit for bit (the skipped
paths add exact zeros).  The bf16-feature layers read the links as float16 codes
(and the hidden layers round them to bf16 pairs for their dot-product transports);
with float32 links the output moves by less than 1e-2 (a rounding flipped here and
there) and stays within the same 2e-2 bar.  The
last layer with its paths split over two waves (the default on small lattices) and
unsplit agree to float32 summation order (1e-5)."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)
WIDTHS = [4, 8, 8, 4]


def _weights(seed):
    return [ls.gaussian_complex((9, WIDTHS[l + 1], WIDTHS[l]), seed + l) for l in range(len(WIDTHS) - 1)]


def _device(W, bf16):
    import torch
    t = torch.from_numpy(np.stack([W.real, W.imag], -1).astype(np.float32)).cuda()
    return (t.to(torch.bfloat16) if bf16 else t).contiguous()


def _bf16_ref(W):
    return (orc.round16(W.real.astype(np.float32), "bf16") + 1j * orc.round16(W.imag.astype(np.float32), "bf16"))


def _oracle(U, dims, v, Ws):
    full = orc.eo_merge(v, np.zeros_like(v), dims)
    out = orc.network_forward(U, orc.spinor_to_features(full), [W.astype(np.complex128) for W in Ws], BC)
    return orc.eo_split(orc.features_to_spinor(out), dims, 0)


def _apply(w, ctx, g, lat, Vh, ws, prec, fin):
    fout = w.new_field(lat, w.EVEN, w.F32)
    widths = (ctypes.c_int * len(WIDTHS))(*WIDTHS)
    ptrs = (ctypes.c_void_p * len(ws))(*[t.data_ptr() for t in ws])
    w.wd_ptnet_apply_even(g.handle, len(ws), widths, ptrs, prec, fin.data_ptr(), fout.data_ptr())
    return fout, w.unpack(ctx, lat, w.EVEN, w.F32, fout, (Vh, 4, 3))


# 6 x 6 x 4 x 10: 720 even sites, 11.25 waves of 64 (a ragged last wave)
@pytest.mark.parametrize("dims", [(6, 6, 4, 10), (8, 4, 4, 6)])
def test_preconditioner_application_matches_oracle(dims, monkeypatch):
    import torch
    from paper_0810_5365_amd import wdirac as w
    X, Y, Z, T = dims
    Vh = X * Y * Z * T // 2
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.7, 5021)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    v = ls.gaussian_complex((Vh, 4, 3), 5023, ls.STREAM_SPINOR)
    fin = w.pack(ctx, lat, w.EVEN, w.F32, v)
    W = _weights(5030)
    # float32 weights: vector units, float32 features
    _, got = _apply(w, ctx, g, lat, Vh, [_device(x, False) for x in W], w.F32, fin)
    assert orc.rel_l2(got, _oracle(U, dims, v, W)) < 1e-5
    # bf16 weights: matrix cores, bf16 hidden features
    wb = [_device(x, True) for x in W]
    ref = _oracle(U, dims, v, [_bf16_ref(x) for x in W])
    f_hf, got_hf = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
    err_hf = orc.rel_l2(got_hf, ref)
    assert 1e-6 < err_hf < 2e-2, err_hf
    # on lattices this small the last layer splits each site group's paths over two waves;
    # unsplit, the same products are summed in another order (float32 accumulation)
    monkeypatch.setenv("WD_PTCONV_SPLIT", "0")
    _, got_one = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
    monkeypatch.delenv("WD_PTCONV_SPLIT")
    assert orc.rel_l2(got_one, got_hf) < 1e-5
    # the bf16-feature layers read the links as float16 codes by default; with float32 links the
    # result moves by the link rounding (2^-11, a bf16 rounding flipped here and there), far
    # less than the bf16 roundings of the features themselves
    monkeypatch.setenv("WD_PTCONV_LINKS32", "1")
    _, got_l32 = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
    monkeypatch.delenv("WD_PTCONV_LINKS32")
    assert orc.rel_l2(got_l32, ref) < 2e-2
    d16 = orc.rel_l2(got_hf, got_l32)
    assert d16 < 1e-2, d16
    # the same with float32 hidden features, with and without the parity skip
    monkeypatch.setenv("WD_PTNET_F32_FEATURES", "1")
    f_32, got_32 = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
    monkeypatch.setenv("WD_PTCONV_PARITY_SKIP", "0")
    f_ns, _ = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
    torch.cuda.synchronize()
    assert orc.rel_l2(got_32, ref) < 2e-2
    assert torch.equal(f_32, f_ns)
    assert not torch.equal(f_hf, f_32)
    g.close()
    ctx.close()


def test_bf16_hidden_features_in_both_wave_orders(monkeypatch):
    """16 x 8 x 4 x 6 (X Y / 2 = 64): the matrix-core layers with bf16 hidden features give
    bit-identical results in the natural and the z-blocked (depth 2) wave order."""
    import torch
    from paper_0810_5365_amd import wdirac as w
    dims = (16, 8, 4, 6)
    Vh = 16 * 8 * 4 * 6 // 2
    ctx = w.Context(0)
    U = ls.gauge_field(dims, 0.7, 5041)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(U)
    lat = w.lattice(dims, BC)
    v = ls.gaussian_complex((Vh, 4, 3), 5043, ls.STREAM_SPINOR)
    fin = w.pack(ctx, lat, w.EVEN, w.F32, v)
    W = _weights(5050)
    wb = [_device(x, True) for x in W]
    outs = []
    for zb in ("0", "2"):
        monkeypatch.setenv("WD_PTCONV_ZB", zb)
        f, got = _apply(w, ctx, g, lat, Vh, wb, w.BF16, fin)
        torch.cuda.synchronize()
        outs.append((f.clone(), got))
    assert torch.equal(outs[0][0], outs[1][0])
    assert orc.rel_l2(outs[1][1], _oracle(U, dims, v, [_bf16_ref(x) for x in W])) < 2e-2
    g.close()
    ctx.close()


def test_preconditioner_application_rejects_bad_input():
    from paper_0810_5365_amd import wdirac as w
    dims = (4, 4, 4, 4)
    ctx = w.Context(0)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(ls.gauge_field(dims, 0.5, 81))
    lat = w.lattice(dims, BC)
    lib = w._raw()
    f = w.new_field(lat, w.EVEN, w.F32)
    o = w.new_field(lat, w.EVEN, w.F32)
    ws = [_device(x, False) for x in _weights(90)]
    ptrs = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ws])
    good = (ctypes.c_int * 4)(*WIDTHS)
    assert lib.wd_ptnet_apply_even(g.handle, 3, good, ptrs, w.F32, f.data_ptr(), f.data_ptr()) == w.WD_EINVAL
    assert lib.wd_ptnet_apply_even(g.handle, 0, good, ptrs, w.F32, f.data_ptr(), o.data_ptr()) == w.WD_EINVAL
    assert lib.wd_ptnet_apply_even(g.handle, 3, good, ptrs, w.F64, f.data_ptr(), o.data_ptr()) == w.WD_EINVAL
    bad = (ctypes.c_int * 4)(2, 8, 8, 4)
    assert lib.wd_ptnet_apply_even(g.handle, 3, bad, ptrs, w.F32, f.data_ptr(), o.data_ptr()) == w.WD_EINVAL
    odd = (ctypes.c_int * 4)(4, 5, 8, 4)
    assert lib.wd_ptnet_apply_even(g.handle, 3, odd, ptrs, w.F32, f.data_ptr(), o.data_ptr()) == w.WD_EUNSUPPORTED
    g.close()
    ctx.close()
