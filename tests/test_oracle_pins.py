"""Pins for the FP64 oracle: each check ties the oracle to something other than
itself -- closed forms, the Clifford algebra, invariants of the Wilson operator,
library routines (scipy's sparse solver, math.fsum, numpy float16, torch's
bfloat16 cast) or brute force -- so a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import lattice_synth as ls
import oracle as orc

BC = (1, 1, 1, -1)
HERE = os.path.dirname(os.path.abspath(__file__))


def spinor(dims, seed):
    return ls.gaussian_spinor(dims, seed)


# ---------------------------------------------------------------------------
# input generator
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(v, 16) for v in r]
        out = ls.philox4x32_10(vals[0:4], vals[4:6])
        assert [int(v) for v in out] == vals[6:10]


def test_generated_links_are_su3_and_third_row_identity():
    U = ls.gauge_field((4, 4, 2, 4), 0.5, 7)
    u = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1.0).max() < 1e-14
    # 12-real reconstruction: row 2 = conj(row0 x row1) holds for SU(3)
    assert np.abs(orc.third_row(u) - u[:, 2, :]).max() < 1e-15 * 10
    # not the trivial field
    assert np.abs(u - eye).max() > 0.1


def test_generated_links_are_exp_of_traceless_hermitian():
    # log of U (principal branch) is i*eps*H with H traceless Hermitian, |eps*H| small
    eps = 0.3
    u = ls.random_su3(64, eps, 99)
    w, v = np.linalg.eig(u)
    assert np.allclose(np.abs(w), 1.0, atol=1e-13)
    phases = np.angle(w)
    assert np.abs(phases.sum(axis=-1)).max() < 1e-12          # traceless generator
    # a Hermitian generator: U is normal, so eigenvectors can be taken unitary
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - np.eye(3)).max() < 1e-14


def test_gaussian_source_statistics():
    s = ls.gaussian_spinor((8, 8, 8, 8), 3)
    assert abs(np.mean(np.abs(s) ** 2) - 1.0) < 0.02
    assert abs(np.mean(s.real ** 2) - 0.5) < 0.02
    assert abs(np.mean(s.real * s.imag)) < 0.02


# ---------------------------------------------------------------------------
# gamma matrices
# ---------------------------------------------------------------------------

def test_gamma_clifford_algebra_and_chirality():
    g = [orc.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.array_equal(g[mu], np.conj(g[mu]).T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.array_equal(ac, 2.0 * (mu == nu) * np.eye(4))
    # DeGrand-Rossi basis: gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 is diag(1, 1, -1, -1)
    assert np.array_equal(orc.gamma5(), np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex))
    # the basis is chiral with real gamma_2, gamma_4 and imaginary gamma_1, gamma_3
    assert np.all(g[1].imag == 0) and np.all(g[3].imag == 0)
    assert np.all(g[0].real == 0) and np.all(g[2].real == 0)


# ---------------------------------------------------------------------------
# free field: closed forms
# ---------------------------------------------------------------------------

def _momentum(dims, n, bc):
    return np.array([2 * np.pi * (n[m] + (0.5 if bc[m] < 0 else 0.0)) / dims[m] for m in range(4)])


def _plane_wave(dims, p, u):
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    return phase[..., None, None] * u[None, None, None, None]


@pytest.mark.parametrize("dagger", [False, True])
def test_free_field_plane_wave(dagger):
    dims = (4, 6, 2, 8)
    U = ls.unit_gauge(dims)
    kappa = 0.137
    u = ls.gaussian_complex((4, 3), 11)
    g = [orc.gamma(mu) for mu in range(4)]
    for n in [(0, 0, 0, 0), (1, 2, 1, 3), (3, 5, 1, 7), (2, 1, 0, 4)]:
        p = _momentum(dims, n, BC)
        psi = _plane_wave(dims, p, u)
        # M(p) = (1 - 2 kappa sum cos p) + 2 i kappa sum gamma sin p ; dagger flips the sine term
        sgn = -1.0 if dagger else 1.0
        Mp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + sgn * 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = _plane_wave(dims, p, Mp @ u)
        got = orc.apply_m(U, psi, kappa, BC, dagger=dagger)
        assert orc.rel_l2(got, expect) < 1e-13


def _dense(op, shape):
    n = int(np.prod(shape))
    cols = []
    for k in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[k] = 1.0
        cols.append(op(e.reshape(shape)).ravel())
    return np.array(cols).T


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 2)])
def test_free_field_spectrum(dims):
    kappa = 0.11
    U = ls.unit_gauge(dims)
    X, Y, Z, T = dims
    A = _dense(lambda v: orc.apply_m(U, v, kappa, BC), (T, Z, Y, X, 4, 3))
    ev = np.linalg.eigvals(A)
    expect = []
    for n in np.ndindex(*dims):
        p = _momentum(dims, n, BC)
        a = 1 - 2 * kappa * np.cos(p).sum()
        b = 2 * kappa * np.sqrt((np.sin(p) ** 2).sum())
        expect += [a + 1j * b] * 6 + [a - 1j * b] * 6
    expect = np.array(expect)
    got = np.sort_complex(np.round(ev, 10))
    exp = np.sort_complex(np.round(expect, 10))
    assert np.abs(got - exp).max() < 1e-9
    # same multiset to high precision: match each expected value to its nearest eigenvalue
    for z in np.unique(np.round(expect, 12)):
        mult_exp = np.sum(np.abs(expect - z) < 1e-10)
        mult_got = np.sum(np.abs(ev - z) < 1e-10)
        assert mult_exp == mult_got


# ---------------------------------------------------------------------------
# general gauge field: invariants
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rough():
    dims = (4, 4, 4, 8)
    return dims, ls.gauge_field(dims, 0.5, 21)


def _g5(psi):
    return np.einsum("st,...tc->...sc", orc.gamma5(), psi)


def test_gamma5_hermiticity(rough):
    dims, U = rough
    psi = spinor(dims, 1)
    kappa = 0.124
    lhs = _g5(orc.apply_m(U, _g5(psi), kappa, BC))
    rhs = orc.apply_m(U, psi, kappa, BC, dagger=True)
    assert orc.rel_l2(lhs, rhs) < 1e-14


def test_adjoint_identity(rough):
    dims, U = rough
    phi, psi = spinor(dims, 2), spinor(dims, 3)
    kappa = 0.124
    a = orc.dot(phi, orc.apply_m(U, psi, kappa, BC))
    b = orc.dot(orc.apply_m(U, phi, kappa, BC, dagger=True), psi)
    assert abs(a - b) < 1e-13 * abs(a)
    # and the adjoint is not trivially the operator itself
    c = orc.dot(orc.apply_m(U, phi, kappa, BC, dagger=False), psi)
    assert abs(c - a) > 1e-3 * abs(a)


def _transform_links(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        Om_fwd = np.roll(Om, -1, axis=ax)
        out[mu] = Om @ U[mu] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    return out


def test_gauge_covariance(rough):
    dims, U = rough
    Om = ls.gauge_transform(dims, 5)
    psi = spinor(dims, 4)
    kappa = 0.124
    UO = _transform_links(U, Om)
    Opsi = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, psi)
    lhs = orc.apply_m(UO, Opsi, kappa, BC)
    rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, orc.apply_m(U, psi, kappa, BC))
    assert orc.rel_l2(lhs, rhs) < 1e-14
    lhs = orc.apply_m(UO, Opsi, kappa, BC, dagger=True)
    rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", Om, orc.apply_m(U, psi, kappa, BC, dagger=True))
    assert orc.rel_l2(lhs, rhs) < 1e-14


def test_parity_structure(rough):
    dims, U = rough
    psi = spinor(dims, 6)
    par = orc.site_parity(dims)
    for p in (0, 1):
        masked = psi * (par == p)[..., None, None]
        out = orc.dhop(U, masked, BC)
        # hopping connects only opposite parities: P_p D_hop P_p = 0
        assert np.abs(out[par == p]).max() == 0.0
        assert np.abs(out[par != p]).max() > 0.1
    # out_parity restriction is the masked full operator
    full = orc.dhop(U, psi, BC)
    for p in (0, 1):
        part = orc.dhop(U, psi, BC, out_parity=p)
        assert np.array_equal(part[par == p], full[par == p])
        assert np.abs(part[par != p]).max() == 0.0


def test_translation_covariance(rough):
    dims, U = rough
    psi = spinor(dims, 7)
    kappa = 0.1
    ref = orc.apply_m(U, psi, kappa, BC)
    # shifts along the periodic spatial directions commute with M
    for ax_lat, ax_U in [(3, 4), (2, 3), (1, 2)]:
        Us = np.roll(U, 1, axis=ax_U)
        ps = np.roll(psi, 1, axis=ax_lat)
        assert np.array_equal(orc.apply_m(Us, ps, kappa, BC), np.roll(ref, 1, axis=ax_lat))


def test_antiperiodic_time_boundary():
    # with U = 1 and a t-constant spinor, only the two time slices at the wrap see a sign flip
    dims = (2, 2, 2, 4)
    U = ls.unit_gauge(dims)
    u = ls.gaussian_complex((4, 3), 3)
    psi = np.broadcast_to(u, (4, 2, 2, 2, 4, 3)).copy()
    per = orc.dhop(U, psi, (1, 1, 1, 1))
    anti = orc.dhop(U, psi, (1, 1, 1, -1))
    g4 = orc.gamma(3)
    diff = per - anti
    # forward hop from t = T-1 carries (1 - g4) * 2u, backward hop into t = 0 carries (1 + g4) * 2u
    assert np.allclose(diff[3], 2 * ((np.eye(4) - g4) @ u), atol=1e-14)
    assert np.allclose(diff[0], 2 * ((np.eye(4) + g4) @ u), atol=1e-14)
    assert np.abs(diff[1:3]).max() == 0.0


def test_single_precision_build_computes_the_same_operator():
    # the FP32 build of the oracle source (timed by the benchmark only) is the same operator
    # to float32 rounding, on both output parities
    dims = (4, 2, 4, 6)
    U = ls.gauge_field(dims, 0.5, 41)
    psi = spinor(dims, 42)
    for par in (0, 1):
        ref = orc.dhop(U, psi, BC, out_parity=par)
        got = orc.dhop_fp32(U, psi, BC, out_parity=par).astype(np.complex128)
        assert 1e-9 < orc.rel_l2(got, ref) < 1e-6


# ---------------------------------------------------------------------------
# even-odd preconditioning (Schur complement)
# ---------------------------------------------------------------------------

def test_eo_split_merge_roundtrip_and_order():
    dims = (4, 2, 2, 4)
    psi = spinor(dims, 8)
    e = orc.eo_split(psi, dims, 0)
    o = orc.eo_split(psi, dims, 1)
    assert e.shape == (32, 4, 3) and o.shape == (32, 4, 3)
    assert np.array_equal(orc.eo_merge(e, o, dims), psi)
    # cb index = lex >> 1 within each parity
    X, Y, Z, T = dims
    par = orc.site_parity(dims).ravel()
    lex = np.arange(X * Y * Z * T)
    for p in (0, 1):
        assert np.array_equal(lex[par == p] >> 1, np.arange(X * Y * Z * T // 2))


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 4)])
def test_eo_schur_solution_matches_sparse_solve(dims):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    U = ls.gauge_field(dims, 0.5, 31)
    kappa = 0.124
    X, Y, Z, T = dims
    shape = (T, Z, Y, X, 4, 3)
    M = sp.csc_matrix(_dense(lambda v: orc.apply_m(U, v, kappa, BC), shape))
    b = spinor(dims, 9)
    x_ref = spla.spsolve(M, b.ravel()).reshape(shape)
    # even-odd route: (1 - kappa^2 D_eo D_oe) x_e = b_e + kappa D_eo b_o ; x_o = b_o + kappa D_oe x_e
    bh = orc.schur_source(U, b, kappa, BC)
    Vh = X * Y * Z * T // 2
    Mh = _dense(lambda v: orc.mhat(U, v, kappa, BC), (Vh, 4, 3))
    x_e = np.linalg.solve(Mh, bh.ravel()).reshape(Vh, 4, 3)
    x = orc.schur_reconstruct(U, x_e, b, kappa, BC)
    assert orc.rel_l2(x, x_ref) < 1e-12
    assert orc.rel_residual(lambda v: orc.apply_m(U, v, kappa, BC), x, b) < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 4), (4, 2, 2, 4)])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("dagger", [False, True])
def test_eo_schur_both_parities_and_daggers_match_sparse_solve(dims, parity, dagger):
    """Each parity's Schur complement, with and without the dagger, solves the full system.

    Block form of M (or M^dagger) over (even, odd) sites: [[1, -k D_eo], [-k D_oe, 1]].
    Eliminating the other parity gives, for parity p with partner q,
        (1 - k^2 D_pq D_qp) x_p = b_p + k D_pq b_q,   x_q = b_q + k D_qp x_p,
    with every hop daggered for M^dagger.  The reference x is scipy's sparse LU solve of
    the full lattice system, so a swapped hop order, a kappa power or a dagger slip in the
    oracle's parity-1 or dagger branch of mhat fails here."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    U = ls.gauge_field(dims, 0.5, 37)
    kappa = 0.124
    X, Y, Z, T = dims
    shape = (T, Z, Y, X, 4, 3)
    Vh = X * Y * Z * T // 2
    M = sp.csc_matrix(_dense(lambda v: orc.apply_m(U, v, kappa, BC, dagger=dagger), shape))
    b = spinor(dims, 11)
    x_ref = spla.spsolve(M, b.ravel()).reshape(shape)
    q = 1 - parity
    hop_pq = orc.d_eo if parity == 0 else orc.d_oe     # q-sites -> p-sites
    hop_qp = orc.d_oe if parity == 0 else orc.d_eo     # p-sites -> q-sites
    b_p, b_q = orc.eo_split(b, dims, parity), orc.eo_split(b, dims, q)
    bh = b_p + kappa * hop_pq(U, b_q, BC, dagger)
    Mh = _dense(lambda v: orc.mhat(U, v, kappa, BC, dagger=dagger, parity=parity), (Vh, 4, 3))
    x_p = np.linalg.solve(Mh, bh.ravel()).reshape(Vh, 4, 3)
    x_q = b_q + kappa * hop_qp(U, x_p, BC, dagger)
    x = orc.eo_merge(x_p, x_q, dims) if parity == 0 else orc.eo_merge(x_q, x_p, dims)
    assert orc.rel_l2(x, x_ref) < 1e-12
    assert orc.rel_residual(lambda v: orc.apply_m(U, v, kappa, BC, dagger=dagger), x, b) < 1e-12
    if not dagger:
        # the normal operator of this parity is the product of the two pinned branches
        Mh_dag = _dense(lambda v: orc.mhat(U, v, kappa, BC, dagger=True, parity=parity), (Vh, 4, 3))
        assert np.abs(Mh_dag - Mh.conj().T).max() < 1e-13
        N = _dense(lambda v: orc.mhat_dag_mhat(U, v, kappa, BC, parity), (Vh, 4, 3))
        assert np.abs(N - Mh.conj().T @ Mh).max() < 1e-12


def test_mhat_adjoint_and_normal_operator(rough):
    dims, U = rough
    X, Y, Z, T = dims
    Vh = X * Y * Z * T // 2
    kappa = 0.124
    a = ls.gaussian_complex((Vh, 4, 3), 1)
    b = ls.gaussian_complex((Vh, 4, 3), 2)
    for parity in (0, 1):
        lhs = orc.dot(a, orc.mhat(U, b, kappa, BC, parity=parity))
        rhs = orc.dot(orc.mhat(U, a, kappa, BC, dagger=True, parity=parity), b)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)
        # M^dag M is Hermitian positive definite
        q = orc.dot(a, orc.mhat_dag_mhat(U, a, kappa, BC, parity))
        assert abs(q.imag) < 1e-12 * abs(q.real) and q.real > 0
    # D_eo^dagger is the adjoint of D_oe
    lhs = orc.dot(a, orc.d_eo(U, b, BC))
    rhs = orc.dot(orc.d_oe(U, a, BC, dagger=True), b)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# ---------------------------------------------------------------------------
# global sums
# ---------------------------------------------------------------------------

def test_dot_and_norm_against_fsum():
    a = ls.gaussian_complex((1000, 12), 1)
    b = ls.gaussian_complex((1000, 12), 2)
    d = orc.dot(a, b)
    prods = np.conj(a.ravel()) * b.ravel()
    assert abs(d.real - math.fsum(prods.real)) < 1e-13 * abs(d)
    assert abs(d.imag - math.fsum(prods.imag)) < 1e-13 * abs(d)
    n = orc.norm2(a)
    assert abs(n - math.fsum((np.abs(a.ravel()) ** 2).tolist())) < 1e-14 * n


# ---------------------------------------------------------------------------
# 16-bit storage codec
# ---------------------------------------------------------------------------

def test_round16_known_values():
    # 1/3 in binary16 is 0x3555 = 0.333251953125; in bfloat16 0x3EAB = 0.333984375
    assert float(orc.round16(np.float32(1 / 3), "f16")) == 0.333251953125
    assert float(orc.round16(np.float32(1 / 3), "bf16")) == 0.333984375
    # ties to even: 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7
    assert float(orc.round16(np.float32(1 + 2.0 ** -8), "bf16")) == 1.0
    assert float(orc.round16(np.float32(1 + 3 * 2.0 ** -8), "bf16")) == 1 + 2 * 2.0 ** -7


def test_bf16_rounding_matches_torch_cast():
    import torch
    x = ls.gaussian_complex((4096,), 5).real.astype(np.float32)
    x[:16] = np.array([1 + k * 2.0 ** -8 for k in range(16)], dtype=np.float32)   # exact ties
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(orc.round16(x, "bf16"), ref)


@pytest.mark.parametrize("kind,ulp", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_spinor_codec_scale_and_error_bound(kind, ulp):
    psi = ls.gaussian_complex((500, 4, 3), 7)
    psi[3] = 0.0
    dec, s, q = orc.quantize_spinor_sites(psi, kind)
    v = np.stack([psi.real, psi.imag], -1).reshape(500, 24).astype(np.float32)
    assert np.array_equal(s, np.abs(v).max(axis=1))
    assert np.abs(q).max() <= 1.0
    # the largest component is stored exactly (code +-1)
    assert np.all(np.abs(q[s > 0]).max(axis=1) == 1.0)
    err = np.abs(np.stack([dec.real, dec.imag], -1).reshape(500, 24) - v)
    assert np.all(err <= (0.5 * ulp + 2.0 ** -23) * s[:, None] + 1e-30)
    assert np.all(dec[3] == 0)


# ---------------------------------------------------------------------------
# parallel-transport convolution
# ---------------------------------------------------------------------------

def _wilson_as_ptconv(kappa):
    g = [orc.gamma(mu) for mu in range(4)]
    W = np.zeros((9, 4, 4), dtype=np.complex128)
    W[0] = np.eye(4)
    for mu in range(4):
        W[1 + mu] = -kappa * (np.eye(4) - g[mu])
        W[5 + mu] = -kappa * (np.eye(4) + g[mu])
    return W


def test_ptconv_with_spin_weights_is_wilson_operator(rough):
    # an independent (numpy-shift) route to M: pins wref.c and the transports together
    dims, U = rough
    kappa = 0.124
    psi = spinor(dims, 12)
    phi = orc.spinor_to_features(psi)
    out = orc.features_to_spinor(orc.ptconv_forward(U, phi, _wilson_as_ptconv(kappa), BC))
    assert orc.rel_l2(out, orc.apply_m(U, psi, kappa, BC)) < 1e-14
    # dagger: swap the projectors
    Wd = _wilson_as_ptconv(kappa)
    Wd[1:5], Wd[5:9] = Wd[5:9].copy(), Wd[1:5].copy()
    out = orc.features_to_spinor(orc.ptconv_forward(U, phi, Wd, BC))
    assert orc.rel_l2(out, orc.apply_m(U, psi, kappa, BC, dagger=True)) < 1e-14


def test_ptconv_identity_and_covariance(rough):
    dims, U = rough
    X, Y, Z, T = dims
    phi = ls.gaussian_complex((3, T, Z, Y, X, 3), 13)
    W = np.zeros((9, 3, 3), dtype=np.complex128)
    W[0] = np.eye(3)
    assert np.array_equal(orc.ptconv_forward(U, phi, W, BC), phi)
    W = ls.gaussian_complex((9, 2, 3), 14)
    Om = ls.gauge_transform(dims, 15)
    UO = _transform_links(U, Om)
    rot = lambda f: np.einsum("tzyxab,ctzyxb->ctzyxa", Om, f)
    lhs = orc.ptconv_forward(UO, rot(phi), W, BC)
    rhs = rot(orc.ptconv_forward(U, phi, W, BC))
    assert orc.rel_l2(lhs, rhs) < 1e-14


def test_ptconv_adjoint_identities(rough):
    dims, U = rough
    X, Y, Z, T = dims
    phi = ls.gaussian_complex((3, T, Z, Y, X, 3), 16)
    chi = ls.gaussian_complex((2, T, Z, Y, X, 3), 17)
    for p in range(9):
        a = orc.dot(chi[:1], orc.transport(U, phi[:1], p, BC))
        b = orc.dot(orc.transport_dagger(U, chi[:1], p, BC), phi[:1])
        assert abs(a - b) < 1e-13 * abs(a)
    W = ls.gaussian_complex((9, 2, 3), 18)
    a = orc.dot(chi, orc.ptconv_forward(U, phi, W, BC))
    b = orc.dot(orc.ptconv_backward_input(U, chi, W, BC), phi)
    assert abs(a - b) < 1e-13 * abs(a)


def test_ptconv_gradients_against_finite_differences():
    dims = (2, 2, 2, 4)
    X, Y, Z, T = dims
    U = ls.gauge_field(dims, 0.7, 41)
    phi = ls.gaussian_complex((2, T, Z, Y, X, 3), 19)
    W = ls.gaussian_complex((9, 3, 2), 20)
    c = ls.gaussian_complex((3, T, Z, Y, X, 3), 21)

    # a non-linear real loss: L = sum |psi|^4 / 4 + Re <c, psi>;  dL/dpsi (torch convention) = |psi|^2 psi + c
    def loss(ph, w):
        ps = orc.ptconv_forward(U, ph, w, BC)
        return float(np.sum(np.abs(ps) ** 4) / 4 + orc.dot(c, ps).real)

    ps = orc.ptconv_forward(U, phi, W, BC)
    gout = np.abs(ps) ** 2 * ps + c
    gW = orc.ptconv_backward_weight(U, phi, gout, BC)
    gin = orc.ptconv_backward_input(U, gout, W, BC)
    h = 1e-5
    # central differences: O(h^2) truncation plus cancellation error ~ eps |L| / h
    slack = 4e-16 * abs(loss(phi, W)) / h
    rng = np.random.default_rng(0)
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in W.shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += unit * h
            Wm[idx] -= unit * h
            fd = (loss(phi, Wp) - loss(phi, Wm)) / (2 * h)
            an = gW[idx].real if part == "re" else gW[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + slack
    for _ in range(12):
        idx = tuple(rng.integers(0, n) for n in phi.shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            pp, pm = phi.copy(), phi.copy()
            pp[idx] += unit * h
            pm[idx] -= unit * h
            fd = (loss(pp, W) - loss(pm, W)) / (2 * h)
            an = gin[idx].real if part == "re" else gin[idx].imag
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + slack
