"""GPU: the allocation-free global sum against the ordinary one.

wd_dot_noalloc keeps its partial sums in a static per-device array instead of a
context's workspace; it runs the same kernels with the same grid, so its result must
equal wd_dot's bit for bit, on two calls in a row (the second on a smaller field, so
stale partials of the first call would show), and match the oracle's float64 dot.
"""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


def _field(dims, subset_full, nrhs, seed):
    X, Y, Z, T = dims
    shape = (T, Z, Y, X, 4, 3) if subset_full else (X * Y * Z * T // 2, 4, 3)
    return ls.gaussian_complex((nrhs,) + shape, seed, ls.STREAM_SPINOR)


# (dims, subset, prec, nrhs): a large field first (1024 workgroups of partials), then smaller
CASES = [((16, 16, 16, 32), "full", "f32", 2), ((4, 4, 4, 4), "even", "f64", 1), ((6, 4, 10, 4), "odd", "bf16", 3),
         ((2, 2, 2, 2), "even", "f16", 1)]


def test_dot_noalloc_matches_dot_on_calls_in_a_row():
    import torch
    from paper_0810_5365_amd import wdirac as w
    ctx = w.Context(0)
    stream = torch.cuda.Stream()
    lib = w._raw()
    for k, (dims, subset, prec, nrhs) in enumerate(CASES):
        sub, p = w.SUBSET_BY_NAME[subset], w.PREC_BY_NAME[prec]
        lat = w.lattice(dims, BC)
        a = _field(dims, sub == w.FULL, nrhs, 100 + k)
        b = _field(dims, sub == w.FULL, nrhs, 200 + k)
        fa = w.pack(ctx, lat, sub, p, a, nrhs)
        fb = w.pack(ctx, lat, sub, p, b, nrhs)
        torch.cuda.synchronize()
        ref = (ctypes.c_double * 2)()
        w.wd_dot(ctx.handle, ctypes.byref(lat), sub, p, nrhs, fa.data_ptr(), fb.data_ptr(), ref)
        for st in (None, stream.cuda_stream):   # the null stream, then a torch stream
            got = (ctypes.c_double * 2)()
            s = lib.wd_dot_noalloc(st, ctypes.byref(lat), sub, p, nrhs, fa.data_ptr(), fb.data_ptr(), got)
            assert s == w.WD_OK, lib.wd_last_error()
            assert (got[0], got[1]) == (ref[0], ref[1]), (dims, prec, tuple(got), tuple(ref))
        # against the oracle's float64 dot of what the packed fields hold
        da = w.unpack(ctx, lat, sub, p, fa, a.shape, nrhs)
        db = w.unpack(ctx, lat, sub, p, fb, b.shape, nrhs)
        d = orc.dot(da, db)
        assert abs(complex(got[0], got[1]) - d) <= 1e-12 * np.sqrt(orc.norm2(da) * orc.norm2(db))
    # bad arguments: nothing runs
    lat = w.lattice((4, 4, 4, 4), BC)
    got = (ctypes.c_double * 2)(7.0, 7.0)
    f = w.new_field(lat, w.EVEN, w.F32)
    assert lib.wd_dot_noalloc(None, ctypes.byref(lat), 9, w.F32, 1, f.data_ptr(), f.data_ptr(), got) == w.WD_EINVAL
    assert lib.wd_dot_noalloc(None, ctypes.byref(lat), w.EVEN, w.F32, 1, None, f.data_ptr(), got) == w.WD_EINVAL
    assert lib.wd_dot_noalloc(None, ctypes.byref(w.lattice((3, 4, 4, 4))), w.EVEN, w.F32, 1, f.data_ptr(),
                              f.data_ptr(), got) == w.WD_ESHAPE
    assert tuple(got) == (7.0, 7.0)
    ctx.close()
