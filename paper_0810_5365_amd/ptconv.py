"""PyTorch autograd wrapper of the HIP parallel-transport convolution.

``PTConvFunction`` forwards to ``wd_ptconv_forward`` / ``wd_ptconv_backward``
(argument marshalling only); ``PTNet`` stacks such layers with weights kept
as float32 master parameters of shape (9, C_out, C_in, 2) -- (re, im) pairs,
so their real-valued gradients are exactly the library's complex gradients
dL/dRe + i dL/dIm -- and stored at 16 bits for the kernels when asked.

Features are flat float32 tensors in the library's packed layout
(``wd_feature_bytes``); a network input is made from a FULL float32 packed
spinor with ``spinor_to_features`` (channel = spin).
"""
import ctypes

import torch

from . import wdirac as w


def weight_storage(W, wprec):
    """float32 (9, C_out, C_in, 2) -> contiguous tensor holding W at wprec."""
    if wprec == w.F32:
        return W.detach().to(torch.float32).contiguous()
    dt = {w.BF16: torch.bfloat16, w.F16: torch.float16}[wprec]
    return W.detach().to(dt).contiguous()


class PTConvFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, W, gauge, cin, cout, wprec, nsamples):
        Ws = weight_storage(W, wprec)
        vol2 = gauge.geom_vh * 2
        out = torch.empty(nsamples * cout * 3 * vol2 * 2, dtype=torch.float32, device=x.device)
        w.wd_ptconv_forward(gauge.handle, cin, cout, wprec, nsamples, Ws.data_ptr(), x.data_ptr(), out.data_ptr())
        ctx.save_for_backward(x, Ws)
        ctx.meta = (gauge, cin, cout, wprec, nsamples)
        return out

    @staticmethod
    def backward(ctx, gout):
        x, Ws = ctx.saved_tensors
        gauge, cin, cout, wprec, nsamples = ctx.meta
        gout = gout.contiguous()
        gin = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gW = torch.empty((9, cout, cin, 2), dtype=torch.float32, device=x.device) if ctx.needs_input_grad[1] else None
        if gin is not None or gW is not None:
            w.wd_ptconv_backward(gauge.handle, cin, cout, wprec, nsamples, Ws.data_ptr(), x.data_ptr(), gout.data_ptr(),
                                 gin.data_ptr() if gin is not None else None,
                                 gW.data_ptr() if gW is not None else None)
        return gin, gW, None, None, None, None, None


def ptconv(x, W, gauge, cin, cout, wprec=w.F32, nsamples=1):
    return PTConvFunction.apply(x, W, gauge, cin, cout, wprec, nsamples)


class PTNet(torch.nn.Module):
    """Linear stack of parallel-transport convolutions (no activation, no bias),
    widths in colour triplets per site, e.g. (4, 8, 8, 4) = 12 -> 24 -> 24 -> 12 complex."""

    def __init__(self, widths=(4, 8, 8, 4), wprec=w.F32, init_scale=None, generator=None, device="cuda"):
        super().__init__()
        self.widths = tuple(widths)
        self.wprec = wprec
        self.weights = torch.nn.ParameterList()
        for cin, cout in zip(widths[:-1], widths[1:]):
            s = init_scale if init_scale is not None else (1.0 / (9 * cin)) ** 0.5
            Wt = torch.randn((9, cout, cin, 2), generator=generator, dtype=torch.float32) * s
            self.weights.append(torch.nn.Parameter(Wt.to(device)))

    def init_identity(self, hop=0.0):
        """Weights that pass the first min(C_in, C_out) channels through (stay path = 1),
        with an optional small amplitude on the hopping paths."""
        with torch.no_grad():
            for Wp in self.weights:
                Wp.zero_()
                n = min(Wp.shape[1], Wp.shape[2])
                for k in range(n):
                    Wp[0, k, k, 0] = 1.0
                if hop:
                    for k in range(n):
                        Wp[1:, k, k, 0] = hop

    def forward(self, x, gauge, nsamples=1):
        for (cin, cout), Wp in zip(zip(self.widths[:-1], self.widths[1:]), self.weights):
            x = ptconv(x, Wp, gauge, cin, cout, self.wprec, nsamples)
        return x

    def storage(self):
        """Per-layer weight tensors at the kernels' precision (for the C solver)."""
        return [weight_storage(Wp, self.wprec) for Wp in self.weights]


def spinor_to_features(ctx, lat, spinor_f32_full, nsamples=1, out=None):
    n = w.feature_bytes(lat, 4, nsamples) // 4
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=spinor_f32_full.device)
    w.wd_spinor_to_features(ctx.handle, ctypes.byref(lat), nsamples, spinor_f32_full.data_ptr(), out.data_ptr())
    return out


def features_to_spinor(ctx, lat, feat, nsamples=1, out=None):
    if out is None:
        out = torch.empty(w.spinor_bytes(lat, w.FULL, w.F32, nsamples), dtype=torch.uint8, device=feat.device)
    w.wd_features_to_spinor(ctx.handle, ctypes.byref(lat), nsamples, feat.data_ptr(), out.data_ptr())
    return out
