"""Python binding of libadct.so: argument marshalling only.

Every function has the name of the C entry point it calls (without the
``adct_`` prefix).  Torch tensors provide device memory and the stream; all
arithmetic runs in the library's HIP kernels.  If the library is missing
this module raises on import of the first call -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadct.so")

OK, PENDING = 0, 1
E_ARG, E_SHAPE, E_DTYPE, E_HIP, E_NOMEM, E_TOO_LARGE, E_STOPPED, E_TIMEOUT, E_NOTFOUND, E_ALIGN = (
    -1, -2, -3, -4, -5, -6, -7, -8, -9, -10)
U8, I16 = 1, 2


class AdctError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {policy_lib().adct_strerror(code).decode()} ({code})")


class Plane(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("reserved", ctypes.c_int32), ("pitch_bytes", ctypes.c_int64)]


class Job(ctypes.Structure):
    _fields_ = [("src", Plane), ("dst", Plane), ("coef", ctypes.c_void_p), ("sse", ctypes.c_void_p)]


class QuantJob(ctypes.Structure):
    _fields_ = [("src", Plane), ("dst", Plane), ("q", ctypes.c_void_p), ("sse", ctypes.c_void_p),
                ("image_height", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("tiles_per_group", ctypes.c_int32), ("groups_per_item", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"tiles_per_group": self.tiles_per_group, "groups_per_item": self.groups_per_item,
                "wgs_per_cu": self.wgs_per_cu}


OP_ZONAL, OP_QUANT, OP_ZIGZAG = 1, 2, 3
XF_PROPOSED, XF_WHT, XF_DCT = 0, 1, 2
KEEP_ZONAL, KEEP_ZIGZAG = 0, 1
SERVE_PERSISTENT, SERVE_PLAIN = 0, 1
SERVE_DMA_ADAPTIVE, SERVE_DMA_BY_SIZE = 0, 1


class ServerCfg(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_int64), ("qp", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_requests", ctypes.c_int32),
                ("auto_release", ctypes.c_int32), ("tiles_per_item", ctypes.c_int32),
                ("wgs_per_cu", ctypes.c_int32), ("idle_polls", ctypes.c_int32),
                ("dma_min_pixels", ctypes.c_int32), ("dma_policy", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("dst", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("sse", ctypes.c_int64), ("t_arrival_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cancelled", ctypes.c_int64), ("in_flight", ctypes.c_int64), ("tiles_completed", ctypes.c_int64),
                ("pool_bytes", ctypes.c_int64), ("pool_high_water", ctypes.c_int64), ("wall_s", ctypes.c_double),
                ("tiles_per_s", ctypes.c_double), ("latency_p50_ms", ctypes.c_double),
                ("latency_p99_ms", ctypes.c_double), ("latency_mean_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("queue_p50_ms", ctypes.c_double),
                ("queue_p99_ms", ctypes.c_double), ("loop_launches", ctypes.c_int64),
                ("dma_copies", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}

_P = ctypes.c_void_p
_PP = ctypes.POINTER(Plane)
_I32, _I64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double

_SIGNATURES = {
    "adct_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "adct_abi_version": (ctypes.c_int, []),
    "adct_constants": (ctypes.c_int, [_P, _P, _P]),
    "adct_quant_tables": (ctypes.c_int, [ctypes.c_int, _P, _P]),
    "adct_psnr": (ctypes.c_int, [_P, _I32, _D, _D, _P]),
    "adct_host_butterfly": (ctypes.c_int, [_I32, _P, _P]),
    "adct_host_butterfly_count": (ctypes.c_int, [_I32, _P, _P, ctypes.POINTER(_I64)]),
    "adct_fwd2d": (ctypes.c_int, [_PP, _P, _P]),
    "adct_inv2d": (ctypes.c_int, [_P, _I64, _P, _P]),
    "adct_scale": (ctypes.c_int, [_P, _I64, _P, _P]),
    "adct_quant": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P]),
    "adct_dequant": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P]),
    "adct_zonal": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P]),
    "adct_zigzag": (ctypes.c_int, [_P, _I64, ctypes.c_int, _P, _P]),
    "adct_zigzag_ranks": (ctypes.c_int, [_P]),
    "adct_round_check": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_I64)]),
    "adct_zigzag_recon": (ctypes.c_int, [_P, ctypes.c_int, _PP, _PP, _I32, _P, _P]),
    "adct_encode_zigzag": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_ssim": (ctypes.c_int, [_PP, _PP, _I32, _P, _P]),
    "adct_compare_encode": (ctypes.c_int, [_PP, _I32, _I32, ctypes.c_int, _PP, _I32, _P, _P]),
    "adct_t8_constants": (ctypes.c_int, [_P, _P, _P]),
    "adct_t8_quant_tables": (ctypes.c_int, [ctypes.c_int, _P, _P]),
    "adct_t8_fwd2d": (ctypes.c_int, [_PP, _P, _P]),
    "adct_t8_inv2d": (ctypes.c_int, [_P, _I64, _P, _P]),
    "adct_t8_encode_zonal": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_t8_encode_quant": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_mixed_encode": (ctypes.c_int, [_PP, ctypes.c_int, _I64, _P, _P, _PP, _I32, _P, _P]),
    "adct_t32_constants": (ctypes.c_int, [_P, _P, _P]),
    "adct_t32_quant_tables": (ctypes.c_int, [ctypes.c_int, _P, _P]),
    "adct_t32_host_butterfly_count": (ctypes.c_int, [_I32, _P, _P, ctypes.POINTER(_I64)]),
    "adct_t32_fwd2d": (ctypes.c_int, [_PP, _P, _P]),
    "adct_t32_inv2d": (ctypes.c_int, [_P, _I64, _P, _P]),
    "adct_t32_encode_zonal": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_t64_constants": (ctypes.c_int, [_P, _P, _P]),
    "adct_t64_quant_tables": (ctypes.c_int, [ctypes.c_int, _P, _P]),
    "adct_t64_host_butterfly_count": (ctypes.c_int, [_I32, _P, _P, ctypes.POINTER(_I64)]),
    "adct_t64_fwd2d": (ctypes.c_int, [_PP, _P, _P]),
    "adct_t64_inv2d": (ctypes.c_int, [_P, _I64, _P, _P]),
    "adct_t64_encode_zonal": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_t64_encode_quant": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_t32_encode_quant": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_check": (ctypes.c_int, [_P]),
    "adct_recon": (ctypes.c_int, [_P, _PP, _P]),
    "adct_sse": (ctypes.c_int, [_PP, _PP, _I32, _P, _P]),
    "adct_fwd2d_quant": (ctypes.c_int, [_PP, ctypes.c_int, _P, _P]),
    "adct_zonal_recon": (ctypes.c_int, [_P, ctypes.c_int, _PP, _PP, _I32, _P, _P]),
    "adct_dequant_recon": (ctypes.c_int, [_P, ctypes.c_int, _PP, _PP, _I32, _P, _P]),
    "adct_encode_zonal": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_encode_quant": (ctypes.c_int, [_PP, ctypes.c_int, _P, _PP, _I32, _P, _P]),
    "adct_encode_quant_planes": (ctypes.c_int, [_P, _I32, ctypes.c_int, _I32, _P]),
    "adct_default_tune": (ctypes.c_int, [ctypes.POINTER(Tune)]),
    "adct_work_queue": (ctypes.c_int, [_P, _I32, _I32, _I32, _P, _I64, ctypes.POINTER(_I64)]),
    "adct_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(Job), _I32, _I32, _I32,
                                         ctypes.POINTER(Tune)]),
    "adct_batch_submit": (ctypes.c_int, [_P, _P]),
    "adct_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(Tune)]),
    "adct_batch_destroy": (ctypes.c_int, [_P]),
    "adct_batch_run_noalloc": (ctypes.c_int, [ctypes.POINTER(Job), _I32, _I32, _I32, ctypes.POINTER(Tune), _P]),
    "adct_autotune": (ctypes.c_int, [_I32, _I32, ctypes.POINTER(Job), _I32, ctypes.c_char_p, _I32,
                                     ctypes.POINTER(Tune), ctypes.POINTER(_D)]),
    "adct_now_ns": (ctypes.c_int64, []),
    "adct_server_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(ServerCfg)]),
    "adct_server_submit": (ctypes.c_int, [_P, _P, _I32, _I32, _I64, _I64, ctypes.POINTER(ctypes.c_uint64)]),
    "adct_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "adct_server_wait_all": (ctypes.c_int, [_P, _I64]),
    "adct_server_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "adct_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "adct_server_stop": (ctypes.c_int, [_P, _I32]),
    "adct_server_destroy": (ctypes.c_int, [_P]),
    "adct_pool_simulate": (ctypes.c_int, [_I64, _P, _I32, _P, ctypes.POINTER(_I64)]),
    "adct_admission_simulate": (ctypes.c_int, [_I64, _I32, _P, _P, _P, _I32, _P]),
    "adct_percentile": (ctypes.c_int, [_P, _I64, _D, ctypes.POINTER(_D)]),
}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libadct.so not built at {LIB_PATH}: run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def lib():
    """The loaded ctypes library (loads it on first use)."""
    return _lib()


# The host policy (status strings, work queue, pool, admission, percentile)
# is plain C++; ADCT_POLICY_LIB may name a CPU-only build of it (the
# sanitizer-instrumented one of the tests), which then serves these calls.
_POLICY_NAMES = ("adct_strerror", "adct_work_queue", "adct_pool_simulate", "adct_admission_simulate",
                 "adct_percentile")
_POLICY = None


def policy_lib():
    global _POLICY
    path = os.environ.get("ADCT_POLICY_LIB")
    if not path:
        return _lib()
    if _POLICY is None:
        pl = ctypes.CDLL(path)
        for name in _POLICY_NAMES:
            res, args = _SIGNATURES[name]
            fn = getattr(pl, name)
            fn.restype = res
            fn.argtypes = args
        _POLICY = pl
    return _POLICY


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise AdctError(rc, where)
    return rc


# ---------------------------------------------------------------- marshalling
def _torch():
    import torch
    return torch


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.uint8:
        return U8
    if t.dtype == torch.int16:
        return I16
    raise AdctError(E_DTYPE, "plane")


def plane(t) -> Plane:
    """Descriptor of a 2D device tensor (rows may be padded: stride(0) is the pitch)."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise AdctError(E_SHAPE, "plane")
    return Plane(t.data_ptr(), _dtype_code(t), t.shape[0], t.shape[1], 0, t.stride(0) * t.element_size())


def _blocks(t, dtype, where):
    torch = _torch()
    if t.dtype != dtype or not t.is_contiguous() or t.numel() % 256:
        raise AdctError(E_ARG, where)
    return t.numel() // 256


def _new_blocks(n, dtype, like):
    return _torch().empty((n, 16, 16), dtype=dtype, device=like.device)


def _nblk_plane(t):
    return (t.shape[0] // 16) * (t.shape[1] // 16)


# ---------------------------------------------------------------- host calls
def strerror(code: int) -> str:
    return _lib().adct_strerror(code).decode()


def abi_version() -> int:
    return _lib().adct_abi_version()


def constants():
    T = np.empty(256, np.int32)
    s = np.empty(16, np.float64)
    W = np.empty(256, np.int32)
    _check(_lib().adct_constants(T.ctypes.data, s.ctypes.data, W.ctypes.data), "constants")
    return T.reshape(16, 16), s, W.reshape(16, 16)


def quant_tables(qp: int):
    qs = np.empty(256, np.float32)
    dqs = np.empty(256, np.float32)
    _check(_lib().adct_quant_tables(qp, qs.ctypes.data, dqs.ctypes.data), "quant_tables")
    return qs.reshape(16, 16), dqs.reshape(16, 16)


def psnr(sse, pixels_per_image: float, peak: float = 255.0) -> np.ndarray:
    sse = np.ascontiguousarray(np.asarray(sse, dtype=np.int64).reshape(-1))
    out = np.empty(sse.shape[0], np.float64)
    _check(_lib().adct_psnr(sse.ctypes.data, sse.shape[0], pixels_per_image, peak, out.ctypes.data), "psnr")
    return out


def round_check(first_bits: int, count: int) -> int:
    """Mismatches of the kernels' rounding against roundf over a range of fp32 bit patterns."""
    n = _I64(0)
    _check(_lib().adct_round_check(first_bits, count, ctypes.byref(n)), "round_check")
    return n.value


def zigzag_ranks() -> np.ndarray:
    """16x16 int32: the scan position of every coefficient, as the kernels use it."""
    r = np.empty(256, np.int32)
    _check(_lib().adct_zigzag_ranks(r.ctypes.data), "zigzag_ranks")
    return r.reshape(16, 16)


def host_butterfly(x, inverse: bool = False, wht: bool = False, t8_halves: bool = False) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(16))
    y = np.empty(16, np.int32)
    if t8_halves:
        which = 4 if inverse else 3
    else:
        which = 2 if wht else (1 if inverse else 0)
    _check(_lib().adct_host_butterfly(which, x.ctypes.data, y.ctypes.data), "host_butterfly")
    return y


def host_butterfly_count(x, inverse: bool = False, wht: bool = False, t8_halves: bool = False):
    """(output, additions): the kernels' butterfly on the host, with every
    addition and subtraction it makes counted."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(16))
    y = np.empty(16, np.int32)
    which = (4 if inverse else 3) if t8_halves else (2 if wht else (1 if inverse else 0))
    n = _I64(0)
    _check(_lib().adct_host_butterfly_count(which, x.ctypes.data, y.ctypes.data, ctypes.byref(n)),
           "host_butterfly_count")
    return y, n.value


# ---------------------------------------------------------------- device calls
def fwd2d(src, coef=None, stream=None):
    torch = _torch()
    if coef is None:
        coef = _new_blocks(_nblk_plane(src), torch.int32, src)
    p = plane(src)
    _check(_lib().adct_fwd2d(ctypes.byref(p), coef.data_ptr(), _stream(stream)), "fwd2d")
    return coef


def fwd2d_quant(src, qp: int, q=None, stream=None):
    torch = _torch()
    if q is None:
        q = _new_blocks(_nblk_plane(src), torch.int16, src)
    p = plane(src)
    _check(_lib().adct_fwd2d_quant(ctypes.byref(p), qp, q.data_ptr(), _stream(stream)), "fwd2d_quant")
    return q


def inv2d(coef, out=None, stream=None):
    torch = _torch()
    n = _blocks(coef, torch.int32, "inv2d")
    if out is None:
        out = _new_blocks(n, torch.int32, coef)
    _check(_lib().adct_inv2d(coef.data_ptr(), n, out.data_ptr(), _stream(stream)), "inv2d")
    return out


def scale(coef, out=None, stream=None):
    torch = _torch()
    n = _blocks(coef, torch.int32, "scale")
    if out is None:
        out = _new_blocks(n, torch.float32, coef)
    _check(_lib().adct_scale(coef.data_ptr(), n, out.data_ptr(), _stream(stream)), "scale")
    return out


def quant(coef, qp: int, q=None, stream=None):
    torch = _torch()
    n = _blocks(coef, torch.int32, "quant")
    if q is None:
        q = _new_blocks(n, torch.int16, coef)
    _check(_lib().adct_quant(coef.data_ptr(), n, qp, q.data_ptr(), _stream(stream)), "quant")
    return q


def dequant(q, qp: int, zfix=None, stream=None):
    torch = _torch()
    n = _blocks(q, torch.int16, "dequant")
    if zfix is None:
        zfix = _new_blocks(n, torch.int32, q)
    _check(_lib().adct_dequant(q.data_ptr(), n, qp, zfix.data_ptr(), _stream(stream)), "dequant")
    return zfix


def zonal(coef, r: int, zfix=None, stream=None):
    torch = _torch()
    n = _blocks(coef, torch.int32, "zonal")
    if zfix is None:
        zfix = _new_blocks(n, torch.int32, coef)
    _check(_lib().adct_zonal(coef.data_ptr(), n, r, zfix.data_ptr(), _stream(stream)), "zonal")
    return zfix


def zigzag(coef, r: int, zfix=None, stream=None):
    torch = _torch()
    n = _blocks(coef, torch.int32, "zigzag")
    if zfix is None:
        zfix = _new_blocks(n, torch.int32, coef)
    _check(_lib().adct_zigzag(coef.data_ptr(), n, r, zfix.data_ptr(), _stream(stream)), "zigzag")
    return zfix


def recon(zfix, dst, stream=None):
    p = plane(dst)
    _check(_lib().adct_recon(zfix.data_ptr(), ctypes.byref(p), _stream(stream)), "recon")
    return dst


def _ref_args(ref, image_height, sse, dst):
    torch = _torch()
    if ref is None:
        return None, 0, None, None
    if image_height is None:
        image_height = dst.shape[0]
    if sse is None:
        sse = torch.empty(dst.shape[0] // image_height, dtype=torch.int64, device=dst.device)
    return plane(ref), image_height, sse, sse.data_ptr()


def zonal_recon(coef, r: int, dst, ref=None, image_height=None, sse=None, stream=None):
    p = plane(dst)
    rp, ih, sse, sp = _ref_args(ref, image_height, sse, dst)
    _check(_lib().adct_zonal_recon(coef.data_ptr(), r, ctypes.byref(p), ctypes.byref(rp) if rp else None,
                                   ih, sp, _stream(stream)), "zonal_recon")
    return sse


def zigzag_recon(coef, r: int, dst, ref=None, image_height=None, sse=None, stream=None):
    p = plane(dst)
    rp, ih, sse, sp = _ref_args(ref, image_height, sse, dst)
    _check(_lib().adct_zigzag_recon(coef.data_ptr(), r, ctypes.byref(p), ctypes.byref(rp) if rp else None,
                                    ih, sp, _stream(stream)), "zigzag_recon")
    return sse


def dequant_recon(q, qp: int, dst, ref=None, image_height=None, sse=None, stream=None):
    p = plane(dst)
    rp, ih, sse, sp = _ref_args(ref, image_height, sse, dst)
    _check(_lib().adct_dequant_recon(q.data_ptr(), qp, ctypes.byref(p), ctypes.byref(rp) if rp else None,
                                     ih, sp, _stream(stream)), "dequant_recon")
    return sse


def _sse_out(src, image_height, sse, want):
    torch = _torch()
    if not want:
        return 0, None, None
    if image_height is None:
        image_height = src.shape[0]
    if sse is None:
        sse = torch.empty(src.shape[0] // image_height, dtype=torch.int64, device=src.device)
    return image_height, sse, sse.data_ptr()


def encode_zonal(src, r: int, dst, coef=None, image_height=None, sse=None, want_sse=True, stream=None):
    """Returns the per-image SSE tensor (or None when want_sse is False)."""
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_encode_zonal(ctypes.byref(ps), r, coef.data_ptr() if coef is not None else None,
                                    ctypes.byref(pd), ih, sp, _stream(stream)), "encode_zonal")
    return sse


def encode_zigzag(src, r: int, dst, coef=None, image_height=None, sse=None, want_sse=True, stream=None):
    """Returns the per-image SSE tensor (or None when want_sse is False)."""
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_encode_zigzag(ctypes.byref(ps), r, coef.data_ptr() if coef is not None else None,
                                     ctypes.byref(pd), ih, sp, _stream(stream)), "encode_zigzag")
    return sse


# ---------------------------------------------------------------- 8-point calls
def t8_constants():
    """(T8 int32 8x8, s8 float64 [8], W8 int32 8x8)."""
    T = np.empty(64, np.int32)
    s = np.empty(8, np.float64)
    W = np.empty(64, np.int32)
    _check(_lib().adct_t8_constants(T.ctypes.data, s.ctypes.data, W.ctypes.data), "t8_constants")
    return T.reshape(8, 8), s, W.reshape(8, 8)


def t8_quant_tables(qp: int):
    qs = np.empty(64, np.float32)
    dqs = np.empty(64, np.float32)
    _check(_lib().adct_t8_quant_tables(qp, qs.ctypes.data, dqs.ctypes.data), "t8_quant_tables")
    return qs.reshape(8, 8), dqs.reshape(8, 8)


def _nblk8(src):
    return (src.shape[0] // 8) * (src.shape[1] // 8)


def t8_fwd2d(src, coef=None, stream=None):
    torch = _torch()
    if coef is None:
        coef = torch.empty((_nblk8(src), 8, 8), dtype=torch.int32, device=src.device)
    p = plane(src)
    _check(_lib().adct_t8_fwd2d(ctypes.byref(p), coef.data_ptr(), _stream(stream)), "t8_fwd2d")
    return coef


def t8_inv2d(coef, out=None, stream=None):
    torch = _torch()
    n = coef.numel() // 64
    if out is None:
        out = torch.empty_like(coef)
    _check(_lib().adct_t8_inv2d(coef.data_ptr(), n, out.data_ptr(), _stream(stream)), "t8_inv2d")
    return out


def t8_encode_zonal(src, r: int, dst, coef=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t8_encode_zonal(ctypes.byref(ps), r, coef.data_ptr() if coef is not None else None,
                                       ctypes.byref(pd), ih, sp, _stream(stream)), "t8_encode_zonal")
    return sse


def t8_encode_quant(src, qp: int, dst, q=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t8_encode_quant(ctypes.byref(ps), qp, q.data_ptr() if q is not None else None,
                                       ctypes.byref(pd), ih, sp, _stream(stream)), "t8_encode_quant")
    return sse


def t32_constants():
    """(T32 int32 32x32, s32 float64 [32], W32 int32 32x32)."""
    T = np.empty(1024, np.int32)
    s = np.empty(32, np.float64)
    W = np.empty(1024, np.int32)
    _check(_lib().adct_t32_constants(T.ctypes.data, s.ctypes.data, W.ctypes.data), "t32_constants")
    return T.reshape(32, 32), s, W.reshape(32, 32)


def t32_quant_tables(qp: int):
    qs = np.empty(1024, np.float32)
    dqs = np.empty(1024, np.float32)
    _check(_lib().adct_t32_quant_tables(qp, qs.ctypes.data, dqs.ctypes.data), "t32_quant_tables")
    return qs.reshape(32, 32), dqs.reshape(32, 32)


def t32_host_butterfly_count(x, inverse: bool = False):
    """(output, additions) of the kernels' 32-point butterfly run on the host."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(32))
    y = np.empty(32, np.int32)
    n = _I64(0)
    _check(_lib().adct_t32_host_butterfly_count(1 if inverse else 0, x.ctypes.data, y.ctypes.data, ctypes.byref(n)),
           "t32_host_butterfly_count")
    return y, n.value


def _nblk32(src):
    return (src.shape[0] // 32) * (src.shape[1] // 32)


def t32_fwd2d(src, coef=None, stream=None):
    torch = _torch()
    if coef is None:
        coef = torch.empty((_nblk32(src), 32, 32), dtype=torch.int32, device=src.device)
    p = plane(src)
    _check(_lib().adct_t32_fwd2d(ctypes.byref(p), coef.data_ptr(), _stream(stream)), "t32_fwd2d")
    return coef


def t32_inv2d(coef, out=None, stream=None):
    torch = _torch()
    n = coef.numel() // 1024
    if out is None:
        out = torch.empty_like(coef)
    _check(_lib().adct_t32_inv2d(coef.data_ptr(), n, out.data_ptr(), _stream(stream)), "t32_inv2d")
    return out


def t32_encode_zonal(src, r: int, dst, coef=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t32_encode_zonal(ctypes.byref(ps), r, coef.data_ptr() if coef is not None else None,
                                        ctypes.byref(pd), ih, sp, _stream(stream)), "t32_encode_zonal")
    return sse


def t32_encode_quant(src, qp: int, dst, q=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t32_encode_quant(ctypes.byref(ps), qp, q.data_ptr() if q is not None else None,
                                        ctypes.byref(pd), ih, sp, _stream(stream)), "t32_encode_quant")
    return sse


def t64_constants():
    """(T64 int32 64x64, s64 float64 [64], W64 int32 64x64)."""
    T = np.empty(4096, np.int32)
    s = np.empty(64, np.float64)
    W = np.empty(4096, np.int32)
    _check(_lib().adct_t64_constants(T.ctypes.data, s.ctypes.data, W.ctypes.data), "t64_constants")
    return T.reshape(64, 64), s, W.reshape(64, 64)


def t64_quant_tables(qp: int):
    qs = np.empty(4096, np.float32)
    dqs = np.empty(4096, np.float32)
    _check(_lib().adct_t64_quant_tables(qp, qs.ctypes.data, dqs.ctypes.data), "t64_quant_tables")
    return qs.reshape(64, 64), dqs.reshape(64, 64)


def t64_host_butterfly_count(x, inverse: bool = False):
    """(output, additions) of the kernels' 64-point butterfly run on the host."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(64))
    y = np.empty(64, np.int32)
    n = _I64(0)
    _check(_lib().adct_t64_host_butterfly_count(1 if inverse else 0, x.ctypes.data, y.ctypes.data, ctypes.byref(n)),
           "t64_host_butterfly_count")
    return y, n.value


def _nblk64(src):
    return (src.shape[0] // 64) * (src.shape[1] // 64)


def t64_fwd2d(src, coef=None, stream=None):
    torch = _torch()
    if coef is None:
        coef = torch.empty((_nblk64(src), 64, 64), dtype=torch.int32, device=src.device)
    p = plane(src)
    _check(_lib().adct_t64_fwd2d(ctypes.byref(p), coef.data_ptr(), _stream(stream)), "t64_fwd2d")
    return coef


def t64_inv2d(coef, out=None, stream=None):
    torch = _torch()
    n = coef.numel() // 4096
    if out is None:
        out = torch.empty_like(coef)
    _check(_lib().adct_t64_inv2d(coef.data_ptr(), n, out.data_ptr(), _stream(stream)), "t64_inv2d")
    return out


def t64_encode_zonal(src, r: int, dst, coef=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t64_encode_zonal(ctypes.byref(ps), r, coef.data_ptr() if coef is not None else None,
                                        ctypes.byref(pd), ih, sp, _stream(stream)), "t64_encode_zonal")
    return sse


def t64_encode_quant(src, qp: int, dst, q=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_t64_encode_quant(ctypes.byref(ps), qp, q.data_ptr() if q is not None else None,
                                        ctypes.byref(pd), ih, sp, _stream(stream)), "t64_encode_quant")
    return sse


def check(stream=None):
    """Waits for `stream` and raises AdctError if its work (or an earlier HIP
    call of this thread) failed."""
    _check(_lib().adct_check(_stream(stream)), "check")


MIXED_MAX_LAMBDA = 1 << 40


def mixed_encode(src, qp: int, lam: int, dst, q=None, split=None, image_height=None, sse=None, want_sse=True,
                 stream=None):
    """Mixed 8/16-point codec: per 16x16 region the coding (one 16x16 block or
    four 8x8 blocks) of lower D + lam * R; returns the per-image SSE."""
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_mixed_encode(ctypes.byref(ps), qp, lam, q.data_ptr() if q is not None else None,
                                    split.data_ptr() if split is not None else None, ctypes.byref(pd), ih, sp,
                                    _stream(stream)), "mixed_encode")
    return sse


def compare_encode(src, transform: int, retention: int, r: int, dst, image_height=None, sse=None, want_sse=True,
                   stream=None):
    """Codec with a comparison transform (XF_PROPOSED / XF_WHT / XF_DCT); returns the per-image SSE."""
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_compare_encode(ctypes.byref(ps), transform, retention, r, ctypes.byref(pd), ih, sp,
                                      _stream(stream)), "compare_encode")
    return sse


def ssim(a, b, image_height=None, out=None, stream=None):
    """Mean SSIM per image of two uint8 planes (float64 device tensor)."""
    torch = _torch()
    if image_height is None:
        image_height = a.shape[0]
    if out is None:
        out = torch.empty(a.shape[0] // image_height, dtype=torch.float64, device=a.device)
    pa, pb = plane(a), plane(b)
    _check(_lib().adct_ssim(ctypes.byref(pa), ctypes.byref(pb), image_height, out.data_ptr(), _stream(stream)),
           "ssim")
    return out


def encode_quant(src, qp: int, dst, q=None, image_height=None, sse=None, want_sse=True, stream=None):
    ps, pd = plane(src), plane(dst)
    ih, sse, sp = _sse_out(src, image_height, sse, want_sse)
    _check(_lib().adct_encode_quant(ctypes.byref(ps), qp, q.data_ptr() if q is not None else None,
                                    ctypes.byref(pd), ih, sp, _stream(stream)), "encode_quant")
    return sse


def encode_quant_planes(jobs, qp: int, block: int = 16, want_sse=True, stream=None):
    """Quantising encoder (block 16: T, 8: T8 on 8x8, 32: T32 on 32x32) over
    several planes in one launch.  jobs: a list of (src, dst, q,
    image_height, sse) with q, image_height and sse optional (q None for all
    jobs or for none; sse allocated when None and want_sse).  Returns the
    list of per-image SSE tensors (None entries when not wanted)."""
    arr = (QuantJob * max(1, len(jobs)))()
    keep, out = [], []
    for i, job in enumerate(jobs):
        src, dst = job[0], job[1]
        q = job[2] if len(job) > 2 else None
        ih = job[3] if len(job) > 3 else None
        sse_t = job[4] if len(job) > 4 else None
        ih, sse_t, sp = _sse_out(src, ih, sse_t, want_sse)
        arr[i] = QuantJob(plane(src), plane(dst), q.data_ptr() if q is not None else None, sp, ih, 0)
        keep.append((src, dst, q, sse_t))
        out.append(sse_t)
    _check(_lib().adct_encode_quant_planes(arr, len(jobs), qp, block, _stream(stream)), "encode_quant_planes")
    return out


def sse(a, b, image_height=None, out=None, stream=None):
    torch = _torch()
    if image_height is None:
        image_height = a.shape[0]
    if out is None:
        out = torch.empty(a.shape[0] // image_height, dtype=torch.int64, device=a.device)
    pa, pb = plane(a), plane(b)
    _check(_lib().adct_sse(ctypes.byref(pa), ctypes.byref(pb), image_height, out.data_ptr(), _stream(stream)),
           "sse")
    return out


# ---------------------------------------------------------------- uneven batches
def default_tune() -> Tune:
    t = Tune()
    _check(_lib().adct_default_tune(ctypes.byref(t)), "default_tune")
    return t


def make_tune(tiles_per_group: int, groups_per_item: int, wgs_per_cu: int) -> Tune:
    return Tune(tiles_per_group, groups_per_item, wgs_per_cu, 0)


def work_queue(tiles_per_job, tiles_per_group: int, groups_per_item: int) -> np.ndarray:
    """Items (job, first tile, tile count) as built by the library, shape (n, 3)."""
    t = np.ascontiguousarray(np.asarray(tiles_per_job, dtype=np.int64).reshape(-1))
    n = _I64(0)
    _check(policy_lib().adct_work_queue(t.ctypes.data, t.shape[0], tiles_per_group, groups_per_item, None, 0,
                                  ctypes.byref(n)), "work_queue")
    items = np.empty((max(n.value, 1), 3), dtype=np.uint32)
    _check(policy_lib().adct_work_queue(t.ctypes.data, t.shape[0], tiles_per_group, groups_per_item, items.ctypes.data,
                                  n.value, ctypes.byref(n)), "work_queue")
    return items[:n.value]


def make_jobs(srcs, dsts, coefs=None, sses=None):
    """A ctypes array of adct_job from lists of device tensors (coef/sse entries may be None)."""
    n = len(srcs)
    arr = (Job * n)()
    for i in range(n):
        c = coefs[i] if coefs is not None else None
        e = sses[i] if sses is not None else None
        arr[i] = Job(plane(srcs[i]), plane(dsts[i]), c.data_ptr() if c is not None else None,
                     e.data_ptr() if e is not None else None)
    return arr


class Batch:
    """One persistent, graph-captured launch over uneven images.  Keeps the
    tensors it was built from alive for its lifetime."""

    def __init__(self, srcs, dsts, op: int, param: int, coefs=None, sses=None, tune: Tune | None = None):
        self._keep = (list(srcs), list(dsts), coefs, sses)
        jobs = make_jobs(srcs, dsts, coefs, sses)
        h = _P()
        _check(_lib().adct_batch_create(ctypes.byref(h), jobs, len(jobs), op, param,
                                        ctypes.byref(tune) if tune is not None else None), "batch_create")
        self._h = h

    def submit(self, stream=None):
        _check(_lib().adct_batch_submit(self._h, _stream(stream)), "batch_submit")

    def info(self):
        tiles, items, t = _I64(0), _I64(0), Tune()
        _check(_lib().adct_batch_info(self._h, ctypes.byref(tiles), ctypes.byref(items), ctypes.byref(t)),
               "batch_info")
        return {"tiles": tiles.value, "items": items.value, "tune": t.as_dict()}

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib().adct_batch_destroy(self._h), "batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_run_noalloc(srcs, dsts, op: int, param: int, coefs=None, sses=None, tune: Tune | None = None,
                      stream=None):
    """One uneven batch coded without any device allocation: the job table
    and work queue live in the library's fixed device array (shared by every
    call on the device; calls must not overlap).  Asynchronous on `stream`:
    the tensors must stay alive until the stream has run it."""
    jobs = make_jobs(srcs, dsts, coefs, sses)
    _check(_lib().adct_batch_run_noalloc(jobs, len(jobs), op, param,
                                         ctypes.byref(tune) if tune is not None else None, _stream(stream)),
           "batch_run_noalloc")


NOALLOC_SCRATCH_BYTES = 16 << 20  # ADCT_NOALLOC_SCRATCH_BYTES


def autotune(srcs, dsts, op: int, param: int, coefs=None, sses=None, cache_path=None, reps: int = 3):
    """(Tune, ms) -- ms is -1.0 when the result came from the cache."""
    jobs = make_jobs(srcs, dsts, coefs, sses)
    t, ms = Tune(), _D(0.0)
    _check(_lib().adct_autotune(op, param, jobs, len(jobs), cache_path.encode() if cache_path else None, reps,
                                ctypes.byref(t), ctypes.byref(ms)), "autotune")
    return t, ms.value


# ---------------------------------------------------------------- serving
def now_ns() -> int:
    return _lib().adct_now_ns()


class Server:
    """Continuous-batching server (persistent device loop) or the plain
    per-request baseline (mode=SERVE_PLAIN).  Submitted host buffers are kept
    referenced until the server is closed."""

    def __init__(self, pool_bytes: int, qp: int = 27, mode: int = SERVE_PERSISTENT, max_inflight: int = 64,
                 max_requests: int = 4096, auto_release: bool = False, tiles_per_item: int = 0,
                 wgs_per_cu: int = 0, idle_polls: int = 0, dma_min_pixels: int = 0,
                 dma_policy: int = 0):
        cfg = ServerCfg(pool_bytes, qp, mode, max_inflight, max_requests, 1 if auto_release else 0, tiles_per_item,
                        wgs_per_cu, idle_polls, dma_min_pixels, dma_policy)
        h = _P()
        _check(_lib().adct_server_create(ctypes.byref(h), ctypes.byref(cfg)), "server_create")
        self._h = h
        self._keep = []

    def submit(self, pixels, arrival_ns: int = -1) -> int:
        """pixels: a 2D uint8 host tensor or numpy array (pinned for asynchronous copies)."""
        if hasattr(pixels, "data_ptr"):
            ptr, (h, w), pitch = pixels.data_ptr(), pixels.shape, pixels.stride(0)
        else:
            ptr, (h, w), pitch = pixels.ctypes.data, pixels.shape, pixels.strides[0]
        t = ctypes.c_uint64(0)
        _check(_lib().adct_server_submit(self._h, ptr, h, w, pitch, arrival_ns, ctypes.byref(t)), "server_submit")
        self._keep.append(pixels)
        return t.value

    def poll(self, ticket: int):
        """(status, Result): status is OK, PENDING, E_STOPPED or E_NOTFOUND."""
        r = Result()
        rc = _lib().adct_server_poll(self._h, ticket, ctypes.byref(r))
        if rc < 0 and rc not in (E_STOPPED, E_NOTFOUND):
            raise AdctError(rc, "server_poll")
        return rc, r

    def wait_all(self, timeout_s: float = 60.0):
        _check(_lib().adct_server_wait_all(self._h, int(timeout_s * 1e9)), "server_wait_all")

    def release(self, ticket: int):
        _check(_lib().adct_server_release(self._h, ticket), "server_release")

    def stats(self) -> dict:
        st = Stats()
        _check(_lib().adct_server_stats(self._h, ctypes.byref(st)), "server_stats")
        return st.as_dict()

    def stop(self, drain: bool = True):
        _check(_lib().adct_server_stop(self._h, 1 if drain else 0), "server_stop")

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib().adct_server_destroy(self._h), "server_destroy")
            self._h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    def __init__(self, ptr: int, shape, typestr: str):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 2}


def device_view(ptr: int, shape, dtype):
    """A torch tensor aliasing server-owned device memory (valid until release)."""
    torch = _torch()
    typestr = {torch.uint8: "|u1", torch.int16: "<i2", torch.int32: "<i4"}[dtype]
    return torch.as_tensor(_DeviceArray(ptr, shape, typestr), device="cuda")


def pool_simulate(capacity: int, ops):
    ops = np.ascontiguousarray(np.asarray(ops, dtype=np.int64))
    out = np.empty(ops.shape[0], dtype=np.int64)
    hw = _I64(0)
    _check(policy_lib().adct_pool_simulate(capacity, ops.ctypes.data, ops.shape[0], out.ctypes.data, ctypes.byref(hw)),
           "pool_simulate")
    return out, hw.value


def admission_simulate(capacity: int, max_inflight: int, arrival, nbytes, hold):
    a = np.ascontiguousarray(np.asarray(arrival, dtype=np.int64))
    b = np.ascontiguousarray(np.asarray(nbytes, dtype=np.int64))
    h = np.ascontiguousarray(np.asarray(hold, dtype=np.int64))
    out = np.empty(a.shape[0], dtype=np.int64)
    _check(policy_lib().adct_admission_simulate(capacity, max_inflight, a.ctypes.data, b.ctypes.data, h.ctypes.data,
                                          a.shape[0], out.ctypes.data), "admission_simulate")
    return out


def percentile(values, p: float) -> float:
    v = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
    out = _D(0.0)
    _check(policy_lib().adct_percentile(v.ctypes.data, v.shape[0], p, ctypes.byref(out)), "percentile")
    return out.value
