"""Property tests of the FP64 oracle over random even lattice shapes (2..8 per
direction), boundary signs, smearing parameters, hopping parameters and seeds:
gamma5-hermiticity, the adjoint identity, gauge covariance, the parity structure
of the hopping term and the 12-real link identity must hold for every draw."""
import numpy as np
from hypothesis import given, settings, strategies as st

import lattice_synth as ls
import oracle as orc

even = st.sampled_from([2, 4, 6, 8])
bcs = st.tuples(*[st.sampled_from([1, -1])] * 4)
SET = settings(max_examples=25, deadline=None, derandomize=True)


def _small(dims):
    return dims[0] * dims[1] * dims[2] * dims[3] <= 1024


def _g5(psi):
    return np.einsum("st,...tc->...sc", orc.gamma5(), psi)


def _transform(U, Om):
    out = np.empty_like(U)
    for mu in range(4):
        ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
        out[mu] = Om @ U[mu] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=ax), -1, -2))
    return out


@SET
@given(dims=st.tuples(even, even, even, even).filter(_small), bc=bcs, eps=st.floats(0.0, 1.0),
       kappa=st.floats(0.05, 0.2), seed=st.integers(1, 10 ** 6))
def test_wilson_operator_identities(dims, bc, eps, kappa, seed):
    U = ls.gauge_field(dims, eps, seed)
    phi, psi = ls.gaussian_spinor(dims, seed + 1), ls.gaussian_spinor(dims, seed + 2)
    Mpsi = orc.apply_m(U, psi, kappa, bc)
    # gamma5 M gamma5 = M^dagger (the dagger computed from its own definition)
    assert orc.rel_l2(_g5(orc.apply_m(U, _g5(psi), kappa, bc)), orc.apply_m(U, psi, kappa, bc, dagger=True)) < 1e-13
    # <phi, M psi> = <M^dagger phi, psi>
    a = orc.dot(phi, Mpsi)
    b = orc.dot(orc.apply_m(U, phi, kappa, bc, dagger=True), psi)
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)
    # gauge covariance
    Om = ls.gauge_transform(dims, seed + 3)
    rot = lambda f: np.einsum("tzyxab,tzyxsb->tzyxsa", Om, f)
    assert orc.rel_l2(orc.apply_m(_transform(U, Om), rot(psi), kappa, bc), rot(Mpsi)) < 1e-13


@SET
@given(dims=st.tuples(even, even, even, even).filter(_small), bc=bcs, seed=st.integers(1, 10 ** 6),
       dagger=st.booleans())
def test_hopping_connects_opposite_parities_only(dims, bc, seed, dagger):
    U = ls.gauge_field(dims, 0.5, seed)
    psi = ls.gaussian_spinor(dims, seed + 1)
    par = orc.site_parity(dims)
    full = orc.dhop(U, psi, bc, dagger)
    for p in (0, 1):
        out = orc.dhop(U, psi * (par == p)[..., None, None], bc, dagger)
        assert np.abs(out[par == p]).max() == 0.0
        # the even-odd blocks are the masked full operator
        np.testing.assert_allclose(out[par != p], full[par != p], rtol=0, atol=1e-13)


@SET
@given(dims=st.tuples(even, even, even, even).filter(_small), eps=st.floats(0.0, 1.5), seed=st.integers(1, 10 ** 6))
def test_generated_links_satisfy_the_twelve_real_identity(dims, eps, seed):
    U = ls.gauge_field(dims, eps, seed)
    u = U.reshape(-1, 3, 3)
    assert np.abs(np.conj(np.cross(u[:, 0], u[:, 1])) - u[:, 2]).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1.0).max() < 1e-13
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - np.eye(3)).max() < 1e-14
