"""FP64 CPU oracle for the Wilson-Dirac hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_0810_5365_amd``) and imports nothing from it; the only module both
sides read is ``lattice_synth``, which draws the seeded inputs.

Everything here is the plain definition, in float64 (complex128), on
canonical lexicographic arrays, without any of the GPU path's rewrites (no spin
projection, no link compression, no structure-of-arrays packing):

* ``dhop`` / ``apply_m``: the Wilson hopping term and M = 1 - kappa*D_hop, from a
  plain C loop over sites with full 4x4 gamma matrices (``wref.c``).
  The operator is the one the paper's Section 4 ("Wilson inverter: main
  features") applies, restricted to even or odd sites.
* ``d_eo`` / ``d_oe`` / ``mhat``: the even-odd preconditioned operator
  1 - kappa^2 D_eo D_oe of the paper's Fig. 2 caption (Section 7), written as
  parity masks around the full-lattice operator.
* ``dot`` / ``norm2``: global sums in double precision (Section 4).
* ``quantize_*``: an independent emulation of the 16-bit storage codec
  (per-site max-norm scale, round-to-nearest-even), and ``third_row`` for the
  12-real link reconstruction the paper describes in Sections 4-5 and 7.
* ``ptconv_*``: parallel-transport convolution layers (the learned
  preconditioner's building block) and their exact gradients, written with
  numpy shifts, independently of ``wref.c``.

Layouts (lattice dims (X, Y, Z, T), all even):
  links    (4, T, Z, Y, X, 3, 3)      complex128
  spinor   (T, Z, Y, X, 4, 3)         complex128, optional leading batch axes
  features (C, T, Z, Y, X, 3)         C colour triplets per site
  half     (Vh, 4, 3)                 one parity's sites in checkerboard order,
                                      cb = lex >> 1, lex = x + X(y + Y(z + Z t))
Parity pins: every function here is pinned by tests/test_oracle_pins.py.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wref.c")
# ORACLE_WREF_LIB / ORACLE_WREF32_LIB name other builds of wref.c to load instead (the
# sanitizer test's)
_LIB_PATH = os.path.join(_HERE, "libwref.so")
_lib = None

BC_DEFAULT = (1, 1, 1, -1)   # periodic in space, antiperiodic in time


_LIB32_PATH = os.path.join(_HERE, "libwref32.so")
_lib32 = None


def build(force=False):
    """Compile wref.c with gcc (never hipcc) into libwref.so, and the same source in single
    precision (-DWREF_FP32; timed by the benchmark's CPU baseline, never checked against)
    into libwref32.so."""
    for path, extra in ((_LIB_PATH, []), (_LIB32_PATH, ["-DWREF_FP32"])):
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared"] + extra + ["-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB_PATH


# ORACLE_WREF_LIB / ORACLE_WREF32_LIB name other builds of wref.c to load instead of the two
# built here (the sanitizer test's).
def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(os.environ.get("ORACLE_WREF_LIB") or _LIB_PATH)
        p = ctypes.c_void_p
        lib.wref_dhop.argtypes = [p, p, p, p, p, ctypes.c_int, ctypes.c_int]
        lib.wref_dhop.restype = None
        lib.wref_gamma.argtypes = [ctypes.c_int, p]
        lib.wref_gamma.restype = None
        lib.wref_num_threads.argtypes = []
        lib.wref_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _load32():
    global _lib32
    if _lib32 is None:
        if not os.path.exists(_LIB32_PATH):
            build()
        lib = ctypes.CDLL(os.environ.get("ORACLE_WREF32_LIB") or _LIB32_PATH)
        p = ctypes.c_void_p
        lib.wref_dhop.argtypes = [p, p, p, p, p, ctypes.c_int, ctypes.c_int]
        lib.wref_dhop.restype = None
        _lib32 = lib
    return _lib32


def dhop_fp32(U, psi, bc=BC_DEFAULT, out_parity=-1):
    """D_hop psi from the single-precision build of the same source (complex64 in and out):
    for timing only, as the CPU counterpart of a single-precision operator."""
    lib = _load32()
    dims = dims_of_links(U)
    U = np.ascontiguousarray(U, dtype=np.complex64)
    psi = np.ascontiguousarray(psi, dtype=np.complex64)
    out = np.empty_like(psi)
    d = np.array(dims, dtype=np.int32)
    b = np.array(bc, dtype=np.int32)
    lib.wref_dhop(d.ctypes.data, b.ctypes.data, U.ctypes.data, psi.ctypes.data, out.ctypes.data, 0, int(out_parity))
    return out


def num_threads():
    return int(_load().wref_num_threads())


def gamma(mu):
    """The 4x4 DeGrand-Rossi gamma matrix for direction mu (0..3 = x, y, z, t)."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().wref_gamma(int(mu), out.ctypes.data)
    return out


def gamma5():
    return gamma(0) @ gamma(1) @ gamma(2) @ gamma(3)


def dims_of_links(U):
    _, T, Z, Y, X = U.shape[:5]
    return (X, Y, Z, T)


# ---------------------------------------------------------------------------
# Wilson operator on the full lattice
# ---------------------------------------------------------------------------

def dhop(U, psi, bc=BC_DEFAULT, dagger=False, out_parity=-1):
    """D_hop psi (or its dagger); leading batch axes of psi are looped over.

    out_parity = 0 / 1 computes only that parity's output sites (others zero).
    """
    lib = _load()
    dims = dims_of_links(U)
    X, Y, Z, T = dims
    U = np.ascontiguousarray(U, dtype=np.complex128)
    site_shape = (T, Z, Y, X, 4, 3)
    if psi.shape[-6:] != site_shape:
        raise ValueError("spinor shape %r does not match links %r" % (psi.shape, U.shape))
    batch = psi.shape[:-6]
    flat = np.ascontiguousarray(psi, dtype=np.complex128).reshape((-1,) + site_shape)
    out = np.empty_like(flat)
    d = np.array(dims, dtype=np.int32)
    b = np.array(bc, dtype=np.int32)
    for k in range(flat.shape[0]):
        lib.wref_dhop(d.ctypes.data, b.ctypes.data, U.ctypes.data, flat[k].ctypes.data,
                      out[k].ctypes.data, int(bool(dagger)), int(out_parity))
    return out.reshape(batch + site_shape)


def apply_m(U, psi, kappa, bc=BC_DEFAULT, dagger=False):
    """M psi = psi - kappa D_hop psi  (M^dagger with dagger=True)."""
    return psi - kappa * dhop(U, psi, bc, dagger)


def apply_mdagm(U, psi, kappa, bc=BC_DEFAULT):
    return apply_m(U, apply_m(U, psi, kappa, bc), kappa, bc, dagger=True)


# ---------------------------------------------------------------------------
# Even-odd (checkerboard) pieces
# ---------------------------------------------------------------------------

def site_parity(dims):
    """Parity (x+y+z+t)&1 of every site, shape (T, Z, Y, X)."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return (x + y + z + t) & 1


_PARITY_INDEX = {}


def parity_sites(dims, parity):
    """Lexicographic indices of the sites of one parity, in checkerboard order."""
    key = (tuple(dims), parity)
    if key not in _PARITY_INDEX:
        _PARITY_INDEX[key] = np.flatnonzero(site_parity(dims).ravel() == parity)
    return _PARITY_INDEX[key]


def eo_split(field, dims, parity, site_ndim=2):
    """Sites of one parity in checkerboard order.

    field: (*batch, T, Z, Y, X, *site) with len(site) == site_ndim
    returns (*batch, Vh, *site).  Within a parity, increasing lexicographic
    order is increasing cb = lex >> 1.
    """
    X, Y, Z, T = dims
    nbatch = field.ndim - 4 - site_ndim
    lead, site = field.shape[:nbatch], field.shape[nbatch + 4:]
    if field.shape[nbatch:nbatch + 4] != (T, Z, Y, X):
        raise ValueError("field shape %r has no lattice axes %r" % (field.shape, (T, Z, Y, X)))
    flat = field.reshape(lead + (X * Y * Z * T,) + site)
    return np.take(flat, parity_sites(dims, parity), axis=nbatch)


def eo_merge(even, odd, dims, site_ndim=2):
    """Inverse of eo_split: two (*batch, Vh, *site) halves -> (*batch, T, Z, Y, X, *site)."""
    X, Y, Z, T = dims
    nbatch = even.ndim - 1 - site_ndim
    lead, site = even.shape[:nbatch], even.shape[nbatch + 1:]
    out = np.empty(lead + (X * Y * Z * T,) + site, dtype=np.result_type(even, odd))
    idx = (slice(None),) * nbatch
    out[idx + (parity_sites(dims, 0),)] = even
    out[idx + (parity_sites(dims, 1),)] = odd
    return out.reshape(lead + (T, Z, Y, X) + site)


def _hop_parity(U, psi_in_half, in_parity, bc, dagger):
    dims = dims_of_links(U)
    zero = np.zeros_like(psi_in_half)
    full = eo_merge(psi_in_half, zero, dims) if in_parity == 0 else eo_merge(zero, psi_in_half, dims)
    out_parity = 1 - in_parity
    res = dhop(U, full, bc, dagger, out_parity=out_parity)
    return eo_split(res, dims, out_parity)


def d_eo(U, psi_o, bc=BC_DEFAULT, dagger=False):
    """D_eo = P_e D_hop P_o: odd-site half spinor -> even-site half spinor."""
    return _hop_parity(U, psi_o, 1, bc, dagger)


def d_oe(U, psi_e, bc=BC_DEFAULT, dagger=False):
    """D_oe = P_o D_hop P_e: even-site half spinor -> odd-site half spinor."""
    return _hop_parity(U, psi_e, 0, bc, dagger)


def mhat(U, psi, kappa, bc=BC_DEFAULT, dagger=False, parity=0):
    """Schur complement on one parity: 1 - kappa^2 D_eo D_oe (parity 0) or
    1 - kappa^2 D_oe D_eo (parity 1); the dagger uses the daggered hops."""
    if parity == 0:
        return psi - kappa * kappa * d_eo(U, d_oe(U, psi, bc, dagger), bc, dagger)
    return psi - kappa * kappa * d_oe(U, d_eo(U, psi, bc, dagger), bc, dagger)


def mhat_dag_mhat(U, psi, kappa, bc=BC_DEFAULT, parity=0):
    return mhat(U, mhat(U, psi, kappa, bc, False, parity), kappa, bc, True, parity)


def schur_source(U, b, kappa, bc=BC_DEFAULT):
    """Even-site right-hand side of the Schur system: b_e + kappa D_eo b_o."""
    dims = dims_of_links(U)
    return eo_split(b, dims, 0) + kappa * d_eo(U, eo_split(b, dims, 1), bc)


def schur_reconstruct(U, x_e, b, kappa, bc=BC_DEFAULT):
    """Full solution from the even half: x_o = b_o + kappa D_oe x_e."""
    dims = dims_of_links(U)
    x_o = eo_split(b, dims, 1) + kappa * d_oe(U, x_e, bc)
    return eo_merge(x_e, x_o, dims)


# ---------------------------------------------------------------------------
# Global sums (double precision)
# ---------------------------------------------------------------------------

def dot(a, b):
    """<a, b> = sum conj(a_i) b_i in complex128."""
    return complex(np.vdot(np.asarray(a, dtype=np.complex128).ravel(), np.asarray(b, dtype=np.complex128).ravel()))


def norm2(a):
    a = np.asarray(a, dtype=np.complex128).ravel()
    return float(np.sum(a.real * a.real + a.imag * a.imag))


def rel_l2(a, ref):
    """||a - ref|| / ||ref|| in float64."""
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.sqrt(norm2(a - ref) / norm2(ref)))


def rel_residual(apply_a, x, b):
    """||b - A x|| / ||b|| recomputed in float64."""
    return float(np.sqrt(norm2(b - apply_a(x)) / norm2(b)))


# ---------------------------------------------------------------------------
# Storage codecs (what the GPU path stores, emulated on the CPU)
# ---------------------------------------------------------------------------

def third_row(U):
    """Row 2 of an SU(3) matrix from rows 0 and 1: conj(row0 x row1)."""
    return np.conj(np.cross(U[..., 0, :], U[..., 1, :]))


def round_f32(x):
    return np.asarray(x).astype(np.float32)


def round_bf16_bits(x_f32):
    """Round float32 values to bfloat16 (round to nearest, ties to even); returns uint16 bits."""
    u = np.asarray(x_f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def round16(x_f32, kind):
    """float32 -> 16-bit (RNE) -> float32."""
    x_f32 = np.asarray(x_f32, dtype=np.float32)
    if kind == "f16":
        return x_f32.astype(np.float16).astype(np.float32)
    if kind == "bf16":
        return bf16_bits_to_f32(round_bf16_bits(x_f32))
    raise ValueError(kind)


def quantize_spinor_sites(psi, kind):
    """16-bit storage of spinor sites with a per-site scale, decoded back.

    psi: complex (..., 4, 3) sites.  Per site: v = float32 of the 24 reals,
    s = max |v_i| (float32), inv = RN(1 / s) (float32), q_i = RNE16(RN(v_i * inv)),
    decoded value RN(q_i * s) (float32 product); s = 0 decodes to zeros.
    Returns (decoded complex128, s float32, q float32-valued codes).
    """
    re = np.stack([psi.real, psi.imag], axis=-1).astype(np.float32)  # (..., 4, 3, 2)
    v = re.reshape(re.shape[:-3] + (24,))
    s = np.max(np.abs(v), axis=-1).astype(np.float32)
    safe = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    inv = (np.float32(1.0) / safe).astype(np.float32)
    q = round16((v * inv[..., None]).astype(np.float32), kind)
    dec = (q * safe[..., None]).astype(np.float32)
    dec = np.where(s[..., None] > 0, dec, np.float32(0.0))
    dec = dec.reshape(re.shape).astype(np.float64)
    return dec[..., 0] + 1j * dec[..., 1], s, q


def quantize_links(U, kind):
    """16-bit link storage: each real entry float32 -> RNE16 (SU(3) entries are bounded by 1)."""
    re = round16(U.real.astype(np.float32), kind).astype(np.float64)
    im = round16(U.imag.astype(np.float32), kind).astype(np.float64)
    return re + 1j * im


def quantize_links_f32(U):
    return U.real.astype(np.float32).astype(np.float64) + 1j * U.imag.astype(np.float32).astype(np.float64)


def reconstruct12(Uq):
    """Keep rows 0, 1 of (already quantised) links and rebuild row 2 = conj(r0 x r1)."""
    out = np.array(Uq, dtype=np.complex128, copy=True)
    out[..., 2, :] = third_row(out)
    return out


# ---------------------------------------------------------------------------
# Parallel-transport convolution (gauge-equivariant layer) and its gradients
# ---------------------------------------------------------------------------
# Paths p = 0 (stay), 1..4 (+mu for mu = x, y, z, t), 5..8 (-mu).
NPATH = 9
_AXIS = {0: 4, 1: 3, 2: 2, 3: 1}   # lattice axis of direction mu in a (C, T, Z, Y, X, 3) array


def _boundary_sign(dims, mu, bc, forward):
    X, Y, Z, T = dims
    L = dims[mu]
    shape = [1, T, Z, Y, X, 1]
    s = np.ones(L)
    if forward:
        s[L - 1] = bc[mu]
    else:
        s[0] = bc[mu]
    view = [1] * 6
    view[_AXIS[mu]] = L
    return s.reshape(view)


def transport(U, phi, p, bc=BC_DEFAULT):
    """(T_p phi)(x): p = 0 identity; 1+mu: U_mu(x) s+ phi(x+mu); 5+mu: U_mu(x-mu)^+ s- phi(x-mu)."""
    if p == 0:
        return phi.copy()
    dims = dims_of_links(U)
    mu = (p - 1) % 4
    ax = _AXIS[mu]
    if p <= 4:
        nb = np.roll(phi, -1, axis=ax) * _boundary_sign(dims, mu, bc, True)
        return np.einsum("tzyxab,ctzyxb->ctzyxa", U[mu], nb)
    Ub = np.roll(U[mu], 1, axis=ax - 1)                       # U_mu(x - mu)
    nb = np.roll(phi, 1, axis=ax) * _boundary_sign(dims, mu, bc, False)
    return np.einsum("tzyxba,ctzyxb->ctzyxa", np.conj(Ub), nb)


def transport_dagger(U, phi, p, bc=BC_DEFAULT):
    """Adjoint of T_p: T_0^+ = T_0, T_{+mu}^+ = T_{-mu}, T_{-mu}^+ = T_{+mu}."""
    if p == 0:
        return phi.copy()
    return transport(U, phi, p + 4 if p <= 4 else p - 4, bc)


def ptconv_forward(U, phi, W, bc=BC_DEFAULT):
    """psi^a(x) = sum_p sum_b W[p, a, b] (T_p phi^b)(x).   W: (9, Cout, Cin)."""
    out = None
    for p in range(NPATH):
        tp = transport(U, phi, p, bc)
        term = np.einsum("ab,bsc->asc", W[p], tp.reshape(tp.shape[0], -1, 3)).reshape((W.shape[1],) + phi.shape[1:])
        out = term if out is None else out + term
    return out


def ptconv_backward_input(U, gout, W, bc=BC_DEFAULT):
    """dL/dphi^b = sum_p T_p^+ sum_a conj(W[p, a, b]) gout^a   (PyTorch complex convention)."""
    gin = None
    for p in range(NPATH):
        mixed = np.einsum("ab,asc->bsc", np.conj(W[p]), gout.reshape(gout.shape[0], -1, 3))
        mixed = mixed.reshape((W.shape[2],) + gout.shape[1:])
        term = transport_dagger(U, mixed, p, bc)
        gin = term if gin is None else gin + term
    return gin


def ptconv_backward_weight(U, phi, gout, bc=BC_DEFAULT):
    """dL/dW[p, a, b] = sum_x sum_c gout^a(x)_c conj((T_p phi^b)(x)_c)."""
    cout, cin = gout.shape[0], phi.shape[0]
    gW = np.zeros((NPATH, cout, cin), dtype=np.complex128)
    g = gout.reshape(cout, -1)
    for p in range(NPATH):
        tp = transport(U, phi, p, bc).reshape(cin, -1)
        gW[p] = g @ np.conj(tp).T
    return gW


def spinor_to_features(psi):
    """(…, T, Z, Y, X, 4, 3) spinor -> (4, T, Z, Y, X, 3) features (spin as channel)."""
    return np.moveaxis(psi, -2, 0)


def features_to_spinor(phi):
    return np.moveaxis(phi, 0, -2)


def network_forward(U, phi, weights, bc=BC_DEFAULT):
    """Linear stack of PT-conv layers (no activation, no bias)."""
    for W in weights:
        phi = ptconv_forward(U, phi, W, bc)
    return phi
