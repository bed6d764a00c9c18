"""Seeded synthetic inputs for the Wilson-Dirac workloads.

The paper benchmarks on gauge fields and volumes it does not list, so every
input here is synthetic: SU(3) links U = exp(i*eps*H) with H a traceless
Hermitian matrix of Gaussian entries, reunitarised, and complex Gaussian
spinors with unit variance per complex entry.  This module holds none of the
operator's arithmetic; it only draws numbers.  Both the FP64 oracle and the GPU
library read its output, so the two sides always start from identical inputs.

Canonical host layouts (numpy complex128, lattice dims given as (X, Y, Z, T)):
  links   : (4, T, Z, Y, X, 3, 3)   U_mu(x)[row, col], mu = x, y, z, t
  spinors : (T, Z, Y, X, 4, 3)      [spin, colour]; a leading nrhs axis if asked
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

# Philox stream ids: one per kind of draw, so fields drawn with the same seed
# for different purposes are independent.
STREAM_LINK = 1
STREAM_SPINOR = 2
STREAM_GAUGE_TRANSFORM = 3
STREAM_MISC = 4


def build(force=False):
    """Compile synth.c with gcc (host only) into libsynth.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        # LATTICE_SYNTH_LIB names another build of synth.c to load instead (the sanitizer test's)
        lib = ctypes.CDLL(os.environ.get("LATTICE_SYNTH_LIB") or _LIB_PATH)
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        ptr = ctypes.c_void_p
        lib.ls_gaussian.argtypes = [u64, u64, u32, dbl, ptr]
        lib.ls_gaussian.restype = None
        lib.ls_su3.argtypes = [u64, dbl, u64, u32, ptr]
        lib.ls_su3.restype = None
        lib.ls_philox4x32_10.argtypes = [ptr, ptr, ptr]
        lib.ls_philox4x32_10.restype = None
        _lib = lib
    return _lib


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block (for the generator's known-answer test)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.ls_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def _check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError("lattice dims must be four even integers >= 2, got %r" % (dims,))
    return dims


def gaussian_complex(shape, seed, stream=STREAM_MISC, var=1.0):
    """Complex Gaussian array with E|z|^2 = var (Re, Im ~ N(0, var/2))."""
    lib = _load()
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.complex128)
    lib.ls_gaussian(n, int(seed), stream, float(var), out.ctypes.data)
    return out.reshape(shape)


def gaussian_spinor(dims, seed, nrhs=None):
    """Complex Gaussian source, unit variance per complex entry.

    Shape (T, Z, Y, X, 4, 3), or (nrhs, T, Z, Y, X, 4, 3) when nrhs is given.
    """
    X, Y, Z, T = _check_dims(dims)
    shape = (T, Z, Y, X, 4, 3) if nrhs is None else (int(nrhs), T, Z, Y, X, 4, 3)
    return gaussian_complex(shape, seed, STREAM_SPINOR)


def random_su3(n, eps, seed, stream=STREAM_MISC):
    """n SU(3) matrices exp(i*eps*H), reunitarised; shape (n, 3, 3)."""
    lib = _load()
    out = np.empty((int(n), 3, 3), dtype=np.complex128)
    lib.ls_su3(int(n), float(eps), int(seed), stream, out.ctypes.data)
    return out


def gauge_field(dims, eps, seed):
    """SU(3) links U_mu(x), shape (4, T, Z, Y, X, 3, 3), drawn in [mu][t][z][y][x] order."""
    X, Y, Z, T = _check_dims(dims)
    V = X * Y * Z * T
    return random_su3(4 * V, eps, seed, STREAM_LINK).reshape(4, T, Z, Y, X, 3, 3)


def unit_gauge(dims):
    """The free field U = 1."""
    X, Y, Z, T = _check_dims(dims)
    U = np.zeros((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gauge_transform(dims, seed, eps=2.0):
    """A random site-dependent SU(3) gauge rotation Omega(x), shape (T, Z, Y, X, 3, 3)."""
    X, Y, Z, T = _check_dims(dims)
    return random_su3(X * Y * Z * T, eps, seed, STREAM_GAUGE_TRANSFORM).reshape(T, Z, Y, X, 3, 3)


def link_seed(config_index, field_index=0):
    """Seed convention: link seed = 1000 * config + field index."""
    return 1000 * int(config_index) + int(field_index)


def source_seed(config_index, field_index=0):
    """Seed convention: source seed = link seed + 500."""
    return link_seed(config_index, field_index) + 500
