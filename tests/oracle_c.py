"""ctypes access to the plain C oracle (test infrastructure)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DIR = os.path.join(os.path.dirname(_HERE), "oracle", "c")
_SO = os.path.join(_DIR, "libadct_oracle.so")
_lib = None


def load():
    global _lib
    if _lib is None:
        src = os.path.join(_DIR, "adct_oracle.c")
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
            subprocess.check_call(["sh", os.path.join(_DIR, "build.sh")])
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_fwd2d_u8.argtypes = [P, I64, I64, I64, P]
        lib.oracle_zonal_recon_u8.argtypes = [P, I64, I64, ctypes.c_int, P, I64, P, I64, P]
        _lib = lib
    return _lib


def threads() -> int:
    return load().oracle_threads()


def set_threads(n: int) -> None:
    load().oracle_set_threads(n)


def fwd2d_u8(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    H, W = img.shape
    coef = np.empty((H // 16 * (W // 16), 16, 16), dtype=np.int64)
    load().oracle_fwd2d_u8(img.ctypes.data, H, W, W, coef.ctypes.data)
    return coef


def zonal_recon_u8(coef: np.ndarray, H: int, W: int, r: int, ref: np.ndarray, image_h: int):
    coef = np.ascontiguousarray(coef, dtype=np.int64)
    out = np.empty((H, W), dtype=np.uint8)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    sse = np.zeros(H // image_h, dtype=np.int64)
    load().oracle_zonal_recon_u8(coef.ctypes.data, H, W, r, out.ctypes.data, W,
                                 ref.ctypes.data, image_h, sse.ctypes.data)
    return out, sse
