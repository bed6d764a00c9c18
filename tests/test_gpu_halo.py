"""GPU: the hopping term on t-slabs of a lattice with half-spinor faces exchanged
between them (device copies standing in for the transfers between devices),
against the FP64 oracle's hopping term on the whole lattice.

Each slab is its own gauge object over its time slices of the global links; the
slab's half fields are the matching contiguous range of the global checkerboard
order (the first slice of every slab is even).  Bars: FP32 <= 1e-5, FP64 <= 1e-12
relative L2, and a single slab exchanging with itself reproduces the ordinary
dslash."""
import ctypes

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def w():
    from paper_0810_5365_amd import wdirac
    return wdirac


@pytest.fixture(scope="module")
def ctx(w):
    c = w.Context(0)
    yield c
    c.close()


def slab_dslash(w, ctx, U, psi_in, dims, nslab, out_even, dagger, prec, recon=12):
    """D_hop (or its dagger) of the global half field psi_in (parity opposite to the
    output) computed slab by slab; returns the global output half field."""
    import torch
    X, Y, Z, T = dims
    Tl = T // nslab
    ldims = (X, Y, Z, Tl)
    lat = w.lattice(ldims, BC)
    vl = X * Y * Z * Tl // 2
    out_sub, in_sub = (w.EVEN, w.ODD) if out_even else (w.ODD, w.EVEN)
    slabs = []
    for r in range(nslab):
        g = w.Gauge(ctx, ldims, BC, recon)
        g.upload(np.ascontiguousarray(U[:, r * Tl:(r + 1) * Tl]))
        fin = w.pack(ctx, lat, in_sub, prec, psi_in[r * vl:(r + 1) * vl])
        ff, fb = w.new_face(lat, prec), w.new_face(lat, prec)
        w.wd_halo_pack(g.handle, in_sub, dagger, prec, fin.data_ptr(), ff.data_ptr(), fb.data_ptr())
        slabs.append((g, fin, ff, fb))
    outs = []
    for r in range(nslab):
        g, fin, _, _ = slabs[r]
        gf = slabs[(r + 1) % nslab][2].clone()        # "received" from the next slab
        gb = slabs[(r - 1) % nslab][3].clone()        # and from the previous one
        sf = BC[3] if r == nslab - 1 else 1.0
        sb = BC[3] if r == 0 else 1.0
        fout = w.new_field(lat, out_sub, prec)
        w.wd_dslash_halo(g.handle, out_sub, dagger, prec, fin.data_ptr(), gf.data_ptr(), gb.data_ptr(), sf, sb,
                         fout.data_ptr())
        outs.append(w.unpack(ctx, lat, out_sub, prec, fout, (vl, 4, 3)))
    torch.cuda.synchronize()
    for g, *_ in slabs:
        g.close()
    return np.concatenate(outs)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dims,nslab", [((4, 6, 2, 8), 2), ((4, 6, 2, 8), 4), ((8, 8, 8, 16), 2), ((6, 4, 4, 12), 3)])
@pytest.mark.parametrize("out_even,dagger", [(True, 0), (False, 1)])
def test_slab_dslash_matches_global_oracle(w, ctx, prec, dims, nslab, out_even, dagger):
    U = ls.gauge_field(dims, 0.5, 71)
    X, Y, Z, T = dims
    psi = ls.gaussian_complex((X * Y * Z * T // 2, 4, 3), 73, ls.STREAM_SPINOR)
    got = slab_dslash(w, ctx, U, psi, dims, nslab, out_even, dagger, w.PREC_BY_NAME[prec])
    ref = orc.d_eo(U, psi, BC, dagger) if out_even else orc.d_oe(U, psi, BC, dagger)
    assert orc.rel_l2(got, ref) < (1e-5 if prec == "f32" else 1e-12)


def test_single_slab_reproduces_the_dslash(w, ctx):
    """One slab that receives its own faces (with the t boundary sign on both) is the
    ordinary antiperiodic-in-t dslash of the whole lattice; 18-real links."""
    dims = (4, 4, 4, 8)
    U = ls.gauge_field(dims, 0.5, 75)
    psi = ls.gaussian_complex((4 * 4 * 4 * 8 // 2, 4, 3), 77, ls.STREAM_SPINOR)
    got = slab_dslash(w, ctx, U, psi, dims, 1, True, 0, w.F32, recon=18)
    lat = w.lattice(dims, BC)
    g = w.Gauge(ctx, dims, BC, 18)
    g.upload(U)
    fin = w.pack(ctx, lat, w.ODD, w.F32, psi)
    fout = w.new_field(lat, w.EVEN, w.F32)
    w.wd_dslash(g.handle, w.EVEN, 0, w.F32, 1, fin.data_ptr(), fout.data_ptr())
    ref = w.unpack(ctx, lat, w.EVEN, w.F32, fout, psi.shape)
    g.close()
    assert orc.rel_l2(got, ref) < 1e-6


def test_slab_entry_points_reject_bad_input(w, ctx):
    dims = (4, 4, 4, 4)
    lat = w.lattice(dims, BC)
    g = w.Gauge(ctx, dims, BC, 12)
    g.upload(ls.gauge_field(dims, 0.5, 79))
    lib = w._raw()
    f = w.new_field(lat, w.ODD, w.F32)
    face = w.new_face(lat, w.F32)
    assert w.face_bytes(lat, w.F32) == 4 * 4 * 4 // 2 * 48 and w.face_bytes(lat, w.F64) == 4 * 4 * 4 // 2 * 96
    assert w.face_bytes(lat, w.BF16) == 0
    p = f.data_ptr()
    assert lib.wd_halo_pack(g.handle, w.FULL, 0, w.F32, p, face.data_ptr(), face.data_ptr()) == w.WD_EINVAL
    assert lib.wd_halo_pack(g.handle, w.ODD, 0, w.BF16, p, face.data_ptr(), face.data_ptr()) == w.WD_EUNSUPPORTED
    assert lib.wd_halo_pack(g.handle, w.ODD, 0, w.F32, p, None, face.data_ptr()) == w.WD_EINVAL
    assert lib.wd_dslash_halo(g.handle, w.EVEN, 0, w.F32, p, face.data_ptr(), face.data_ptr(), 1.0, 1.0,
                              p) == w.WD_EINVAL
    w.wd_gauge_fix_temporal(g.handle, None)
    out = w.new_field(lat, w.EVEN, w.F32)
    assert lib.wd_dslash_halo(g.handle, w.EVEN, 0, w.F32, p, face.data_ptr(), face.data_ptr(), 1.0, 1.0,
                              out.data_ptr()) == w.WD_EUNSUPPORTED
    g.close()
