"""The C ABI without a GPU: the library loads, exports every declared entry
point, its host-side constants agree with the oracle, the kernels' own
butterfly code (run on the host) computes T x and T^T X, and invalid
arguments are rejected before anything is launched."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import adct_oracle as O
from paper_1606_07414_amd import adct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(adct_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = adct.lib()
    names = _declared_functions()
    assert len(names) >= 17
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert _declared_functions() <= set(adct._SIGNATURES)


def test_abi_version():
    assert adct.abi_version() == 1


def test_constants_match_oracle():
    T, s, W = adct.constants()
    assert np.array_equal(T, O.transform_matrix())
    assert np.array_equal(s, O.scaling_vector())
    assert np.array_equal(W, O.zonal_weights())


@pytest.mark.parametrize("qp", list(range(0, 64)))
def test_quant_tables_match_oracle_bit_exact(qp):
    qs, dqs = adct.quant_tables(qp)
    oqs, odqs = O.quant_tables(qp)
    assert np.array_equal(qs.view(np.uint32), oqs.view(np.uint32))
    assert np.array_equal(dqs.view(np.uint32), odqs.view(np.uint32))


def test_quant_tables_reject_bad_qp():
    with pytest.raises(adct.AdctError):
        adct.quant_tables(64)
    with pytest.raises(adct.AdctError):
        adct.quant_tables(-1)


def test_kernel_butterflies_on_host_basis_and_random():
    T = O.transform_matrix()
    for k in range(16):
        e = np.zeros(16, np.int32)
        e[k] = 1
        assert np.array_equal(adct.host_butterfly(e), T[:, k])
        assert np.array_equal(adct.host_butterfly(e, inverse=True), T[k, :])
    rng = np.random.default_rng(1606)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(10000, 16)):
        assert np.array_equal(adct.host_butterfly(x), T @ x)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(2000, 16)):
        assert np.array_equal(adct.host_butterfly(x, inverse=True), T.T @ x)


def test_psnr_host():
    out = adct.psnr([0, 100, 256], 100)
    assert out[0] == math.inf
    assert out[1] == pytest.approx(20 * math.log10(255), rel=1e-15)
    assert out[2] == pytest.approx(O.psnr(256, 100), rel=1e-15)
    with pytest.raises(adct.AdctError):
        adct.psnr([-1], 100)


def test_strerror():
    assert adct.strerror(0) == "ok"
    assert "16" in adct.strerror(adct.E_SHAPE)
    assert adct.strerror(12345) == "unknown status"


# ---- argument validation (fails before any launch, so no GPU is needed) ----
def _plane(ptr, dtype, h, w, pitch):
    return adct.Plane(ptr, dtype, h, w, 0, pitch)


FAKE = 0x10000  # never dereferenced: every case below fails validation


@pytest.mark.parametrize("h,w,pitch,dtype,code", [
    (0, 16, 16, adct.U8, adct.E_SHAPE),
    (16, 0, 16, adct.U8, adct.E_SHAPE),
    (24, 16, 16, adct.U8, adct.E_SHAPE),
    (16, 24, 32, adct.U8, adct.E_SHAPE),
    (16, 32, 16, adct.U8, adct.E_SHAPE),       # pitch < width
    (16, 16, 16, adct.I16, adct.E_SHAPE),      # pitch < 2 * width
    (16, 16, 24, adct.U8, adct.E_ALIGN),       # pitch not a multiple of 16
    (16, 16, 16, 7, adct.E_DTYPE),
])
def test_fwd2d_rejects_bad_planes(h, w, pitch, dtype, code):
    p = _plane(FAKE, dtype, h, w, pitch)
    assert adct.lib().adct_fwd2d(ctypes.byref(p), FAKE, None) == code


def test_rejects_null_and_misaligned():
    lib = adct.lib()
    p = _plane(FAKE, adct.U8, 16, 16, 16)
    assert lib.adct_fwd2d(None, FAKE, None) == adct.E_ARG
    assert lib.adct_fwd2d(ctypes.byref(p), None, None) == adct.E_ARG
    assert lib.adct_fwd2d(ctypes.byref(p), FAKE + 4, None) == adct.E_ALIGN
    q = _plane(FAKE + 8, adct.U8, 16, 16, 16)
    assert lib.adct_fwd2d(ctypes.byref(q), FAKE, None) == adct.E_ALIGN
    assert lib.adct_inv2d(FAKE, -1, FAKE, None) == adct.E_ARG
    assert lib.adct_quant(FAKE, 1, 64, FAKE, None) == adct.E_ARG
    assert lib.adct_dequant(FAKE, 1, -1, FAKE, None) == adct.E_ARG
    assert lib.adct_zonal(FAKE, 1, 17, FAKE, None) == adct.E_ARG
    assert lib.adct_zonal_recon(FAKE, -1, ctypes.byref(p), None, 0, None, None) == adct.E_ARG


def test_empty_block_arrays_are_noops():
    lib = adct.lib()
    # nblk == 0 launches nothing and succeeds, even without a device
    assert lib.adct_inv2d(FAKE, 0, FAKE, None) == adct.OK
    assert lib.adct_scale(FAKE, 0, FAKE, None) == adct.OK
    assert lib.adct_quant(FAKE, 0, 27, FAKE, None) == adct.OK
    assert lib.adct_dequant(FAKE, 0, 27, FAKE, None) == adct.OK
    assert lib.adct_zonal(FAKE, 0, 4, FAKE, None) == adct.OK


def test_recon_reference_rules():
    lib = adct.lib()
    d = _plane(FAKE, adct.U8, 32, 16, 16)
    r_bad = _plane(FAKE, adct.U8, 16, 16, 16)
    # ref and sse must come together
    assert lib.adct_zonal_recon(FAKE, 4, ctypes.byref(d), ctypes.byref(d), 16, None, None) == adct.E_ARG
    # ref shape must match dst
    assert lib.adct_zonal_recon(FAKE, 4, ctypes.byref(d), ctypes.byref(r_bad), 16, FAKE, None) == adct.E_SHAPE
    # image height must divide the plane and be a multiple of 16
    assert lib.adct_zonal_recon(FAKE, 4, ctypes.byref(d), ctypes.byref(d), 24, FAKE, None) == adct.E_SHAPE
    assert lib.adct_zonal_recon(FAKE, 4, ctypes.byref(d), ctypes.byref(d), 48, FAKE, None) == adct.E_SHAPE
    assert lib.adct_sse(ctypes.byref(d), ctypes.byref(r_bad), 16, FAKE, None) == adct.E_SHAPE
