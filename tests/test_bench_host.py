"""Host-side pieces of bench.py: the refusal of more than one GPU, and the plaquette
it reports beside each solve (unit links, gauge invariance, and the values the
link generator gives at the benchmark's smearing parameters)."""
import os
import subprocess
import sys

import numpy as np

import bench
import lattice_synth as ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def test_plaquette_of_unit_links_is_one():
    U = np.broadcast_to(np.eye(3, dtype=complex), (4, 4, 2, 4, 6, 3, 3)).copy()
    assert abs(bench.plaquette(U) - 1.0) < 1e-15


def _random_su3(shape, rng):
    a = rng.normal(size=shape + (3, 3)) + 1j * rng.normal(size=shape + (3, 3))
    q, r = np.linalg.qr(a)
    q = q * (np.diagonal(r, axis1=-2, axis2=-1) / np.abs(np.diagonal(r, axis1=-2, axis2=-1)))[..., None, :]
    return q / np.linalg.det(q)[..., None, None] ** (1.0 / 3.0)


def test_plaquette_is_gauge_invariant():
    """U_mu(x) -> O(x) U_mu(x) O(x + mu)^dag leaves every plaquette unchanged."""
    rng = np.random.default_rng(5)
    U = ls.gauge_field((4, 6, 2, 4), 0.5, 17)
    O = _random_su3(U.shape[1:5], rng)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    V = np.stack([O @ U[mu] @ np.roll(O, -1, axis[mu]).conj().swapaxes(-1, -2) for mu in range(4)])
    assert abs(bench.plaquette(V) - bench.plaquette(U)) < 1e-13


def test_plaquette_of_a_single_twisted_link():
    """One x-link set to a diagonal phase matrix diag(e^{i a}, e^{-i a}, 1), all others unit:
    the four plaquettes that contain it (planes xy, xz, xt, one each side) each hold
    (1/3) Re tr = (2 cos a + 1) / 3, the rest 1."""
    dims = (4, 4, 4, 4)
    U = np.broadcast_to(np.eye(3, dtype=complex), (4,) + dims + (3, 3)).copy()
    a = 0.7
    U[0, 1, 2, 3, 1] = np.diag([np.exp(1j * a), np.exp(-1j * a), 1.0])
    nplaq = 6 * 4 ** 4
    want = ((nplaq - 6) + 6 * (2 * np.cos(a) + 1) / 3) / nplaq
    assert abs(bench.plaquette(U) - want) < 1e-15


def test_plaquette_tracks_the_smearing_parameter():
    """Average plaquettes of generated links at eps = 0.3, 0.5, 0.6, 0.7 on 8^4 sit near
    0.61, 0.24, 0.12, 0.05 (the values the benchmark's fields are quoted with)."""
    for eps, want in ((0.3, 0.61), (0.5, 0.24), (0.6, 0.12), (0.7, 0.05)):
        assert abs(bench.plaquette(ls.gauge_field((8, 8, 8, 8), eps, 6001)) - want) < 0.01
