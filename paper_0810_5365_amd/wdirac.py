"""ctypes binding for libwdirac (argument marshalling only).

Every function here forwards to the C ABI declared in include/wdirac.h under
the same name; all computation runs in the library's HIP kernels.  PyTorch is
used only to own device memory (uint8 tensors sized with wd_spinor_bytes)
and to supply the HIP stream.  If libwdirac.so is missing this module raises
at import: there is no fallback path.
"""
import ctypes
import sys
import os

import numpy as np
# torch first: its bundled HIP runtime must be the one the process loads, so
# that libwdirac.so (NEEDED libamdhip64.so.7) binds to it instead of pulling a
# second runtime copy from /opt/rocm that would not see the device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwdirac.so")

WD_OK, WD_EINVAL, WD_ESHAPE, WD_ENOMEM, WD_EHIP, WD_ENOCONV, WD_ENAN, WD_EUNSUPPORTED = range(8)
F64, F32, F16, BF16 = 0, 1, 2, 3
FULL, EVEN, ODD = 0, 1, 2
RECON_12, RECON_18 = 12, 18
PREC_NAMES = {F64: "f64", F32: "f32", F16: "f16", BF16: "bf16"}
PREC_BY_NAME = {v: k for k, v in PREC_NAMES.items()}
SUBSET_BY_NAME = {"full": FULL, "even": EVEN, "odd": ODD}


class WdLattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("bc", ctypes.c_int * 4)]


class WdSolverParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("sloppy", ctypes.c_int),
                ("delta", ctypes.c_double), ("pure_sloppy", ctypes.c_int)]


class WdSolverInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("operator_applies", ctypes.c_int),
                ("status", ctypes.c_int), ("true_resid", ctypes.c_double), ("true_resid_M", ctypes.c_double),
                ("seconds", ctypes.c_double), ("cycles", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double), ("hops", ctypes.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class WdBatchItem(ctypes.Structure):
    _fields_ = [("gauge", ctypes.c_void_p), ("out_subset", ctypes.c_int), ("dagger", ctypes.c_int),
                ("nrhs", ctypes.c_int), ("in_", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class WdError(RuntimeError):
    def __init__(self, fn, status, detail):
        self.status = status
        super().__init__("%s -> %s: %s" % (fn, _lib.wd_status_string(status).decode(), detail))


_V, _I, _D, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_P = ctypes.POINTER
# name: (restype, argtypes); restype int means a wd_status that is checked
_PROTOS = {
    "wd_abi_version": (_I, []),
    "wd_status_string": (ctypes.c_char_p, [_I]),
    "wd_last_error": (ctypes.c_char_p, []),
    "wd_context_create": ("status", [_I, _V, _P(_V)]),
    "wd_context_set_stream": ("status", [_V, _V]),
    "wd_context_destroy": ("status", [_V]),
    "wd_gauge_create": ("status", [_V, _P(WdLattice), _I, _P(_V)]),
    "wd_gauge_upload": ("status", [_V, _V, _I]),
    "wd_gauge_prepare": ("status", [_V, _I]),
    "wd_gauge_bytes": (_S, [_V, _I]),
    "wd_gauge_destroy": ("status", [_V]),
    "wd_gauge_fix_temporal": ("status", [_V, _V]),
    "wd_spinor_bytes": (_S, [_P(WdLattice), _I, _I, _I]),
    "wd_plane_stride": (ctypes.c_longlong, [_P(WdLattice)]),
    "wd_spinor_pack": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _V]),
    "wd_spinor_unpack": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _V]),
    "wd_spinor_convert": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _I, _V]),
    "wd_dslash": ("status", [_V, _I, _I, _I, _I, _V, _V]),
    "wd_dslash_xpay": ("status", [_V, _I, _I, _I, _I, _V, _V, _D, _D, _V]),
    "wd_apply_M": ("status", [_V, _D, _I, _I, _I, _I, _V, _V]),
    "wd_apply_MdagM": ("status", [_V, _D, _I, _I, _I, _V, _V]),
    "wd_dot": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _V, _P(_D)]),
    "wd_norm2": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _P(_D)]),
    "wd_dot_noalloc": ("status", [_V, _P(WdLattice), _I, _I, _I, _V, _V, _P(_D)]),
    "wd_caxpy": ("status", [_V, _P(WdLattice), _I, _I, _I, _D, _D, _V, _V]),
    "wd_cg_solve": ("status", [_V, _D, _I, _P(WdSolverParams), _V, _V, _P(WdSolverInfo)]),
    "wd_wilson_solve": ("status", [_V, _D, _P(WdSolverParams), _V, _V, _P(WdSolverInfo)]),
    "wd_feature_bytes": (_S, [_P(WdLattice), _I, _I]),
    "wd_feature_pack": ("status", [_V, _P(WdLattice), _I, _I, _V, _V]),
    "wd_feature_unpack": ("status", [_V, _P(WdLattice), _I, _I, _V, _V]),
    "wd_spinor_to_features": ("status", [_V, _P(WdLattice), _I, _V, _V]),
    "wd_features_to_spinor": ("status", [_V, _P(WdLattice), _I, _V, _V]),
    "wd_ptconv_forward": ("status", [_V, _I, _I, _I, _I, _V, _V, _V]),
    "wd_ptconv_backward": ("status", [_V, _I, _I, _I, _I, _V, _V, _V, _V, _V]),
    "wd_batch_create": ("status", [_V, _I, _P(WdBatchItem), _I, _P(_V)]),
    "wd_batch_run": ("status", [_V]),
    "wd_batch_info": ("status", [_V, _P(ctypes.c_longlong), _P(_I)]),
    "wd_batch_shape": ("status", [_V, _P(_I), _P(_I), _P(_I)]),
    "wd_batch_destroy": ("status", [_V]),
    "wd_device_copy": ("status", [_V, _V, _V, _S]),
    "wd_bicgstab_solve": ("status", [_V, _D, _P(WdSolverParams), _V, _V, _P(WdSolverInfo)]),
    "wd_fgmres_solve": ("status", [_V, _D, _P(WdSolverParams), _I, _I, _P(_I), _P(_V), _I, _V, _V, _P(WdSolverInfo)]),
    "wd_ptnet_apply_even": ("status", [_V, _I, _P(_I), _P(_V), _I, _V, _V]),
    "wd_autotune_dslash": ("status", [_V, _I, _I, ctypes.c_char_p]),
    "wd_tune_save": ("status", [_V, ctypes.c_char_p]),
    "wd_tune_load": ("status", [_V, ctypes.c_char_p]),
    "wd_tune_get": (_I, [_V, ctypes.c_char_p, _P(_I)]),
    "wd_tune_get_n": (_I, [_V, ctypes.c_char_p, _P(_I), _I]),
    "wd_face_bytes": (_S, [_P(WdLattice), _I]),
    "wd_halo_pack": ("status", [_V, _I, _I, _I, _V, _V, _V]),
    "wd_dslash_halo": ("status", [_V, _I, _I, _I, _V, _V, _V, _D, _D, _V]),
}

_lib = None
ABI_VERSION = 5   # the structures above match include/wdirac.h at this version


def _raw():
    """The loaded CDLL (raises if the library is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwdirac.so is not built (%s); run `python -m paper_0810_5365_amd.build`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(lib, name)
            f.restype = _I if res == "status" else res
            f.argtypes = args
        if lib.wd_abi_version() != ABI_VERSION:
            raise ImportError("%s has ABI version %d, this binding expects %d; rebuild it"
                              % (LIB_PATH, lib.wd_abi_version(), ABI_VERSION))
        _lib = lib
    return _lib


def exported_symbols():
    return list(_PROTOS)


def _checked(name):
    f = getattr(_raw(), name)

    def call(*args, ok=(WD_OK,)):
        s = f(*args)
        if s not in ok:
            raise WdError(name, s, _lib.wd_last_error().decode())
        return s
    call.__name__ = name
    return call


_raw()
for _name, (_res, _args) in _PROTOS.items():
    globals()[_name] = _checked(_name) if _res == "status" else getattr(_lib, _name)


# ---------------------------------------------------------------------------
# small conveniences (still marshalling only)
# ---------------------------------------------------------------------------

def lattice(dims, bc=(1, 1, 1, -1)):
    lat = WdLattice()
    for d in range(4):
        lat.dims[d] = int(dims[d])
        lat.bc[d] = int(bc[d])
    return lat


def _ptr(t):
    """Device (or host) address of a torch tensor or numpy array."""
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


class Context:
    """A library context bound to a device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        wd_context_create(int(device), ctypes.c_void_p(stream), ctypes.byref(h))
        self.handle = h
        self.device = device

    def set_stream(self, stream):
        wd_context_set_stream(self.handle, ctypes.c_void_p(stream))

    def close(self):
        if self.handle is not None:
            wd_context_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be going away: the process
        # releases the device memory itself, so nothing is called into the library then
        # (the check is bound at definition: module globals may already be None by then)
        if self.handle is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Gauge:
    def __init__(self, ctx, dims, bc=(1, 1, 1, -1), recon=RECON_12):
        self.ctx = ctx
        self.dims = tuple(dims)
        self.bc = tuple(bc)
        self.lat = lattice(dims, bc)
        self.recon = recon
        self.geom_vh = int(np.prod(self.dims)) // 2
        h = ctypes.c_void_p()
        wd_gauge_create(ctx.handle, ctypes.byref(self.lat), int(recon), ctypes.byref(h))
        self.handle = h

    def upload(self, links):
        """links: numpy complex128 (4, T, Z, Y, X, 3, 3) on the host, or a float64 torch tensor on the device."""
        if isinstance(links, np.ndarray):
            arr = np.ascontiguousarray(links, dtype=np.complex128)
            wd_gauge_upload(self.handle, ctypes.c_void_p(arr.ctypes.data), 0)
        else:
            wd_gauge_upload(self.handle, ctypes.c_void_p(links.data_ptr()), 1)

    def prepare(self, prec):
        wd_gauge_prepare(self.handle, int(prec))

    def close(self):
        if self.handle is not None:
            wd_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be going away: the process
        # releases the device memory itself, so nothing is called into the library then
        # (the check is bound at definition: module globals may already be None by then)
        if self.handle is None or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def spinor_bytes(lat, subset, prec, nrhs=1):
    return int(wd_spinor_bytes(ctypes.byref(lat), int(subset), int(prec), int(nrhs)))


def plane_stride(lat):
    return int(wd_plane_stride(ctypes.byref(lat)))


def new_field(lat, subset, prec, nrhs=1, device=0):
    """An uninitialised packed device field (torch uint8 tensor)."""
    import torch
    n = spinor_bytes(lat, subset, prec, nrhs)
    if n == 0:
        raise ValueError("bad field description")
    return torch.empty(n, dtype=torch.uint8, device="cuda:%d" % device)


def face_bytes(lat, prec):
    return int(wd_face_bytes(ctypes.byref(lat), int(prec)))


def new_face(lat, prec, device=0):
    """An uninitialised face buffer of a t-slab (torch uint8 tensor)."""
    import torch
    n = face_bytes(lat, prec)
    if n == 0:
        raise ValueError("bad face description")
    return torch.empty(n, dtype=torch.uint8, device="cuda:%d" % device)


def _check_field(t, lat, subset, prec, nrhs):
    need = spinor_bytes(lat, subset, prec, nrhs)
    got = t.numel() * t.element_size()
    if got < need:
        raise ValueError("field buffer holds %d bytes, needs %d" % (got, need))


def _canon_reals(lat, subset, nrhs):
    """float64 count of a canonical spinor field (nrhs x sites x 4 x 3 complex)."""
    v = int(np.prod(list(lat.dims)))
    return int(nrhs) * (v if int(subset) == FULL else v // 2) * 24


def _check_canon(n, lat, subset, nrhs):
    need = _canon_reals(lat, subset, nrhs)
    if n != need:
        raise ValueError("canonical field holds %d reals, the lattice, subset and nrhs need %d" % (n, need))


def pack(ctx, lat, subset, prec, canon, nrhs=1):
    """canonical complex (numpy, host) or float64 (torch, device) -> new packed device field."""
    import torch
    if isinstance(canon, np.ndarray):
        canon = torch.from_numpy(np.ascontiguousarray(canon, dtype=np.complex128).view(np.float64)).to(
            "cuda:%d" % ctx.device)
    _check_canon(canon.numel() * canon.element_size() // 8, lat, subset, nrhs)
    out = new_field(lat, subset, prec, nrhs, ctx.device)
    wd_spinor_pack(ctx.handle, ctypes.byref(lat), int(subset), int(prec), int(nrhs), ctypes.c_void_p(canon.data_ptr()),
                   ctypes.c_void_p(out.data_ptr()))
    return out


def unpack(ctx, lat, subset, prec, packed, shape, nrhs=1):
    """packed device field -> numpy complex128 of the given canonical shape."""
    import torch
    _check_field(packed, lat, subset, prec, nrhs)
    n = int(np.prod(shape)) * 2
    _check_canon(n, lat, subset, nrhs)
    canon = torch.empty(n, dtype=torch.float64, device="cuda:%d" % ctx.device)
    wd_spinor_unpack(ctx.handle, ctypes.byref(lat), int(subset), int(prec), int(nrhs), ctypes.c_void_p(packed.data_ptr()),
                     ctypes.c_void_p(canon.data_ptr()))
    torch.cuda.current_stream(ctx.device).synchronize()
    return canon.cpu().numpy().view(np.complex128).reshape(shape)


def feature_bytes(lat, channels, nsamples=1):
    return int(wd_feature_bytes(ctypes.byref(lat), int(channels), int(nsamples)))


def pack_features(ctx, lat, canon, channels, nsamples=1):
    """canonical complex (nsamples, C, T, Z, Y, X, 3) on the host -> packed float32 device features."""
    import torch
    c = torch.from_numpy(np.ascontiguousarray(canon, dtype=np.complex128).view(np.float64)).to("cuda:%d" % ctx.device)
    if c.numel() != int(nsamples) * int(channels) * int(np.prod(list(lat.dims))) * 6:
        raise ValueError("canonical features hold %d reals, need %d" % (
            c.numel(), int(nsamples) * int(channels) * int(np.prod(list(lat.dims))) * 6))
    out = torch.empty(feature_bytes(lat, channels, nsamples) // 4, dtype=torch.float32, device="cuda:%d" % ctx.device)
    wd_feature_pack(ctx.handle, ctypes.byref(lat), int(channels), int(nsamples), c.data_ptr(), out.data_ptr())
    return out


def unpack_features(ctx, lat, packed, shape, channels, nsamples=1):
    import torch
    n = int(np.prod(shape)) * 2
    if n != int(nsamples) * int(channels) * int(np.prod(list(lat.dims))) * 6:
        raise ValueError("feature shape %s does not match %d samples of %d channels" % (shape, nsamples, channels))
    canon = torch.empty(n, dtype=torch.float64, device="cuda:%d" % ctx.device)
    wd_feature_unpack(ctx.handle, ctypes.byref(lat), int(channels), int(nsamples), packed.data_ptr(), canon.data_ptr())
    torch.cuda.current_stream(ctx.device).synchronize()
    return canon.cpu().numpy().view(np.complex128).reshape(shape)


def dslash_key(dims, prec, recon, nrhs, dagger, xpay):
    """Tuning-table key of one dslash kernel variant."""
    return "dslash:%dx%dx%dx%d:p%d:r%d:n%d:d%d:x%d" % (tuple(dims) + (prec, recon, nrhs, int(dagger), int(xpay)))


def tune_get(ctx, key):
    out = (ctypes.c_int * 7)()
    if wd_tune_get_n(ctx.handle, key.encode(), out, 7):
        return {"block": out[0], "remap": out[1], "nt": out[2], "pf": out[3], "rhs_inner": out[4], "zb": out[5],
                "mfma": out[6]}
    return None


def solver_params(tol=1e-10, maxiter=10000, sloppy=F32, delta=-1.0, pure_sloppy=False):
    p = WdSolverParams()
    p.tol = tol
    p.maxiter = maxiter
    p.sloppy = int(sloppy)
    p.delta = delta
    p.pure_sloppy = int(bool(pure_sloppy))
    return p
