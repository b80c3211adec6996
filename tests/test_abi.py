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
    assert adct.abi_version() == 2


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


def test_int16_levels_fit_from_qp4_on():
    # The fused quantising encoders saturate levels to int16 only where a
    # level can leave int16.  |Y[u][v]| <= d_u d_v max|x| since T's entries
    # are 0 and +-1, so with int16 samples within [-2047, 2047] the largest
    # level magnitude is max over (u, v) of d_u d_v 2047 qs[u][v] (rounded):
    # below 32767 from QP 4 on, above it below QP 4.  Checked on the
    # library's own fp32 tables; uint8 samples never come close.
    T, _, _ = adct.constants()
    d = (T.astype(np.int64) ** 2).sum(axis=1)
    for qp in range(64):
        qs, _ = adct.quant_tables(qp)
        top = float((np.outer(d, d) * qs.astype(np.float64)).max())
        assert (top * 2047 < 32767) == (qp >= 4), qp
        assert top * 255 < 8000, qp
    # the bound is reached: an all-2047 tile has DC = 256 * 2047
    assert float(adct.quant_tables(4)[0][0, 0]) * 256 * 2047 == pytest.approx(32752, rel=1e-6)


def test_t8_levels_never_leave_int16():
    # The 8-point quantising codecs store levels without saturation: with
    # |Y8[u][v]| <= d_u d_v 2047 (int16 samples within [-2047, 2047]) the
    # largest level is below 26000 at every QP, on the library's own tables.
    T8 = adct.t8_constants()[0]
    d = (T8.astype(np.int64) ** 2).sum(axis=1)
    for qp in range(64):
        qs8, _ = adct.t8_quant_tables(qp)
        assert float((np.outer(d, d) * qs8.astype(np.float64)).max()) * 2047 < 26000, qp


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


def test_kernel_butterflies_count_the_paper_additions(golden_dir):
    """The kernels' own dataflows (the templates the GPU instantiates), run
    with a value type that counts additions: Table 1's 44 for T (and its
    transpose), 64 for the WHT, Section 2.1's 14 for T8 (per half)."""
    import json
    import os
    tab = json.load(open(os.path.join(golden_dir, "table1_complexity.json")))
    T = O.transform_matrix()
    rng = np.random.default_rng(44)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(50, 16)):
        y, n = adct.host_butterfly_count(x)
        assert n == tab["proposed"]["add"] == 44 and np.array_equal(y, T @ x)
        y, n = adct.host_butterfly_count(x, inverse=True)
        assert n == 44 and np.array_equal(y, T.T @ x)
        y, n = adct.host_butterfly_count(x, wht=True)
        assert n == tab["competitor_additions"]["wht"]
        for inv in (False, True):
            y, n = adct.host_butterfly_count(x, inverse=inv, t8_halves=True)
            assert n == 2 * tab["t8_additions"]
            assert np.array_equal(y, adct.host_butterfly(x, inverse=inv, t8_halves=True))
    assert adct.lib().adct_host_butterfly_count(5, FAKE, FAKE, None) == adct.E_ARG


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
    # an empty array may be a null pointer (what an empty device tensor gives)
    assert lib.adct_inv2d(None, 0, None, None) == adct.OK
    assert lib.adct_scale(None, 0, None, None) == adct.OK
    assert lib.adct_quant(None, 0, 27, None, None) == adct.OK
    assert lib.adct_dequant(None, 0, 27, None, None) == adct.OK
    assert lib.adct_zonal(None, 0, 4, None, None) == adct.OK
    assert lib.adct_zigzag(None, 0, 150, None, None) == adct.OK
    assert lib.adct_t8_inv2d(None, 0, None, None) == adct.OK
    # the other arguments are still checked, and a null pointer with blocks is not accepted
    assert lib.adct_quant(None, 0, 64, None, None) == adct.E_ARG
    assert lib.adct_zonal(None, 0, 17, None, None) == adct.E_ARG
    assert lib.adct_inv2d(None, 1, FAKE, None) == adct.E_ARG
    assert lib.adct_inv2d(FAKE, 1, None, None) == adct.E_ARG
    assert lib.adct_t8_inv2d(None, 1, FAKE, None) == adct.E_ARG


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


# ---- host work-queue construction (no GPU) ----
def test_work_queue_small_exact():
    items = adct.work_queue([5, 0, 33], tiles_per_group=8, groups_per_item=2)
    assert items.tolist() == [[0, 0, 5], [2, 0, 16], [2, 16, 16], [2, 32, 1]]


def test_work_queue_covers_every_tile_once():
    rng = np.random.default_rng(4)
    tiles = rng.integers(1, 3000, size=200)
    for tpg, gpi in [(8, 1), (16, 4), (32, 64)]:
        items = adct.work_queue(tiles, tpg, gpi).astype(np.int64)
        span = tpg * gpi
        assert np.all(items[:, 2] >= 1) and np.all(items[:, 2] <= span)
        assert np.all(items[:, 1] % span == 0)  # items start on whole groups
        for j in range(len(tiles)):
            mine = items[items[:, 0] == j]
            covered = np.zeros(tiles[j], dtype=np.int64)
            for _, first, cnt in mine:
                covered[first:first + cnt] += 1
            assert np.all(covered == 1)
        assert np.all(np.diff(items[:, 0]) >= 0)  # job order


def test_work_queue_errors():
    lib = adct.policy_lib()
    n = ctypes.c_int64(0)
    t = np.array([10, 20], dtype=np.int64)
    assert lib.adct_work_queue(t.ctypes.data, 2, 0, 1, None, 0, ctypes.byref(n)) == adct.E_ARG
    assert lib.adct_work_queue(t.ctypes.data, 2, 16, 0, None, 0, ctypes.byref(n)) == adct.E_ARG
    bad = np.array([-1], dtype=np.int64)
    assert lib.adct_work_queue(bad.ctypes.data, 1, 16, 1, None, 0, ctypes.byref(n)) == adct.E_ARG
    out = np.zeros(3, dtype=np.uint32)
    assert lib.adct_work_queue(t.ctypes.data, 2, 16, 1, out.ctypes.data, 1, ctypes.byref(n)) == adct.E_TOO_LARGE
    assert n.value == 3  # 10 tiles -> 1 item, 20 tiles -> 2 items of at most 16


def test_default_tune_and_batch_arg_checks():
    t = adct.default_tune()
    assert t.tiles_per_group in (8, 16, 32) and t.groups_per_item >= 1 and t.wgs_per_cu >= 1
    lib = adct.lib()
    h = ctypes.c_void_p()
    jobs = (adct.Job * 1)()
    jobs[0] = adct.Job(adct.Plane(FAKE, adct.U8, 24, 16, 0, 16), adct.Plane(FAKE, adct.U8, 24, 16, 0, 16), None, None)
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_ZONAL, 8, None) == adct.E_SHAPE
    jobs[0] = adct.Job(adct.Plane(FAKE, adct.U8, 16, 16, 0, 16), adct.Plane(FAKE, adct.I16, 16, 16, 0, 32), None, None)
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_ZONAL, 8, None) == adct.E_SHAPE
    jobs[0] = adct.Job(adct.Plane(FAKE, adct.U8, 16, 16, 0, 16), adct.Plane(FAKE, adct.U8, 16, 16, 0, 16), None, None)
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_ZONAL, 17, None) == adct.E_ARG
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_QUANT, 64, None) == adct.E_ARG
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, 9, 8, None) == adct.E_ARG
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 0, adct.OP_ZONAL, 8, None) == adct.E_ARG
    bad = adct.make_tune(12, 1, 1)
    # a bad tuning is rejected before any device work
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_ZONAL, 8, ctypes.byref(bad)) in (adct.E_ARG, adct.E_HIP)
    assert lib.adct_batch_submit(None, None) == adct.E_ARG
    assert lib.adct_batch_destroy(None) == adct.E_ARG


# ---- zig-zag retention and SSIM (no GPU) ----
def test_zigzag_ranks_match_oracle():
    from oracle import image_experiment as E
    assert np.array_equal(adct.zigzag_ranks(), E.zigzag_index())


def test_zigzag_and_ssim_argument_checks():
    lib = adct.lib()
    p = _plane(FAKE, adct.U8, 32, 32, 32)
    q = _plane(FAKE, adct.I16, 32, 32, 64)
    assert lib.adct_zigzag(FAKE, 1, 257, FAKE, None) == adct.E_ARG
    assert lib.adct_zigzag(FAKE, 1, -1, FAKE, None) == adct.E_ARG
    assert lib.adct_zigzag(FAKE, 0, 150, FAKE, None) == adct.OK
    assert lib.adct_zigzag_recon(FAKE, 300, ctypes.byref(p), None, 0, None, None) == adct.E_ARG
    assert lib.adct_encode_zigzag(ctypes.byref(p), -2, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert lib.adct_encode_zigzag(ctypes.byref(p), 10, None, ctypes.byref(q), 32, None, None) == adct.E_SHAPE
    assert lib.adct_ssim(ctypes.byref(q), ctypes.byref(q), 32, FAKE, None) == adct.E_DTYPE
    small = _plane(FAKE, adct.U8, 16, 32, 32)
    assert lib.adct_ssim(ctypes.byref(p), ctypes.byref(small), 16, FAKE, None) == adct.E_SHAPE
    assert lib.adct_ssim(ctypes.byref(p), ctypes.byref(p), 24, FAKE, None) == adct.E_SHAPE
    assert lib.adct_ssim(ctypes.byref(p), ctypes.byref(p), 32, FAKE + 4, None) == adct.E_ALIGN
    assert lib.adct_ssim(ctypes.byref(p), ctypes.byref(p), 32, None, None) == adct.E_ARG
    h = ctypes.c_void_p()
    jobs = (adct.Job * 1)()
    jobs[0] = adct.Job(adct.Plane(FAKE, adct.U8, 16, 16, 0, 16), adct.Plane(FAKE, adct.U8, 16, 16, 0, 16), None, None)
    assert lib.adct_batch_create(ctypes.byref(h), jobs, 1, adct.OP_ZIGZAG, 257, None) == adct.E_ARG


# ---- 8-point calls (no GPU) ----
def test_t8_constants_and_tables_match_oracle():
    from oracle import t8 as E8
    T, s, W = adct.t8_constants()
    assert np.array_equal(T, E8.transform_matrix_8())
    assert np.array_equal(s, E8.scaling_vector_8())
    assert np.array_equal(W, E8.zonal_weights_8())
    for qp in range(64):
        qs, dqs = adct.t8_quant_tables(qp)
        oqs, odqs = E8.quant_tables_8(qp)
        assert np.array_equal(qs.view(np.uint32), oqs.view(np.uint32)), qp
        assert np.array_equal(dqs.view(np.uint32), odqs.view(np.uint32)), qp


def test_t8_argument_checks():
    lib = adct.lib()
    p = _plane(FAKE, adct.U8, 24, 40, 48)
    odd = _plane(FAKE, adct.U8, 20, 40, 48)
    assert lib.adct_t8_fwd2d(ctypes.byref(odd), FAKE, None) == adct.E_SHAPE
    assert lib.adct_t8_fwd2d(ctypes.byref(p), FAKE + 8, None) == adct.E_ALIGN
    assert lib.adct_t8_fwd2d(ctypes.byref(p), None, None) == adct.E_ARG
    assert lib.adct_t8_encode_zonal(ctypes.byref(p), 9, None, ctypes.byref(p), 24, None, None) == adct.E_ARG
    assert lib.adct_t8_encode_zonal(ctypes.byref(p), 4, None, ctypes.byref(p), 12, FAKE, None) == adct.E_SHAPE
    assert lib.adct_t8_encode_quant(ctypes.byref(p), 64, None, ctypes.byref(p), 24, None, None) == adct.E_ARG
    assert lib.adct_t8_inv2d(FAKE, -1, FAKE, None) == adct.E_ARG
    assert lib.adct_t8_inv2d(FAKE, 0, FAKE, None) == adct.OK
    # u8 rows need 8-byte alignment, int16 rows 16
    assert lib.adct_t8_fwd2d(ctypes.byref(_plane(FAKE + 8, adct.U8, 8, 8, 8)), None, None) == adct.E_ARG
    assert lib.adct_t8_fwd2d(ctypes.byref(_plane(FAKE + 4, adct.U8, 8, 8, 8)), FAKE, None) == adct.E_ALIGN
    assert lib.adct_t8_fwd2d(ctypes.byref(_plane(FAKE + 8, adct.I16, 8, 8, 16)), FAKE, None) == adct.E_ALIGN
    assert lib.adct_t8_fwd2d(ctypes.byref(_plane(FAKE, adct.I16, 8, 8, 24)), FAKE, None) == adct.E_ALIGN
    assert lib.adct_t8_quant_tables(64, None, None) == adct.E_ARG


def test_kernel_rounding_is_round_half_away_for_every_fp32():
    # every finite fp32 whose rounded value fits an int32, both signs
    # (bit patterns 0 .. 0x4F000000 are |x| < 2^31)
    total = 0
    for sign in (0, 0x80000000):
        start = sign
        end = sign + 0x4F000000
        step = 1 << 28
        for b in range(start, end, step):
            total += adct.round_check(b, min(step, end - b))
    assert total == 0


def test_compare_argument_checks():
    lib = adct.lib()
    p = _plane(FAKE, adct.U8, 32, 32, 32)
    assert lib.adct_compare_encode(ctypes.byref(p), 3, 0, 4, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert lib.adct_compare_encode(ctypes.byref(p), 1, 2, 4, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert lib.adct_compare_encode(ctypes.byref(p), 2, 0, 17, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert lib.adct_compare_encode(ctypes.byref(p), 2, 1, 257, ctypes.byref(p), 32, None, None) == adct.E_ARG
    q = _plane(FAKE, adct.U8, 16, 32, 32)
    assert lib.adct_compare_encode(ctypes.byref(p), 1, 0, 4, ctypes.byref(q), 32, None, None) == adct.E_SHAPE


def test_kernel_wht_butterfly_on_host():
    from oracle import comparison as CMP
    H = CMP.wht_matrix()
    for k in range(16):
        e = np.zeros(16, np.int32)
        e[k] = 1
        assert np.array_equal(adct.host_butterfly(e, wht=True), H[:, k])
    rng = np.random.default_rng(16)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(5000, 16)):
        assert np.array_equal(adct.host_butterfly(x, wht=True), H @ x)
    assert adct.lib().adct_host_butterfly(5, np.zeros(16, np.int32).ctypes.data,
                                          np.zeros(16, np.int32).ctypes.data) == adct.E_ARG


def test_kernel_t8_butterflies_on_host():
    from oracle import t8 as E8
    T8 = E8.transform_matrix_8()
    rng = np.random.default_rng(1608)
    for x in rng.integers(-(1 << 20), 1 << 20, size=(3000, 16)):
        want = np.concatenate([T8 @ x[:8], T8 @ x[8:]])
        assert np.array_equal(adct.host_butterfly(x, t8_halves=True), want)
        want_t = np.concatenate([T8.T @ x[:8], T8.T @ x[8:]])
        assert np.array_equal(adct.host_butterfly(x, inverse=True, t8_halves=True), want_t)
    for k in range(16):
        e = np.zeros(16, np.int32)
        e[k] = 1
        col = adct.host_butterfly(e, t8_halves=True)
        assert np.array_equal(col[8 * (k // 8):8 * (k // 8) + 8], T8[:, k % 8])
        assert not col[8 * (1 - k // 8):8 * (1 - k // 8) + 8].any()
    assert adct.lib().adct_host_butterfly(5, FAKE, FAKE) == adct.E_ARG


def test_mixed_argument_checks():
    lib = adct.lib()
    p = _plane(FAKE, adct.I16, 32, 48, 96)
    u8 = _plane(FAKE, adct.U8, 32, 48, 48)
    small = _plane(FAKE, adct.I16, 16, 48, 96)
    f = lib.adct_mixed_encode
    assert f(None, 27, 5, None, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert f(ctypes.byref(p), 27, 5, None, None, ctypes.byref(u8), 32, None, None) == adct.E_SHAPE
    assert f(ctypes.byref(p), 27, 5, None, None, ctypes.byref(small), 32, None, None) == adct.E_SHAPE
    assert f(ctypes.byref(p), 27, -1, None, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert f(ctypes.byref(p), 27, adct.MIXED_MAX_LAMBDA + 1, None, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert f(ctypes.byref(p), 64, 5, None, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert f(ctypes.byref(p), -1, 5, None, None, ctypes.byref(p), 32, None, None) == adct.E_ARG
    assert f(ctypes.byref(p), 27, 5, FAKE + 8, None, ctypes.byref(p), 32, None, None) == adct.E_ALIGN
    assert f(ctypes.byref(p), 27, 5, None, None, ctypes.byref(p), 24, FAKE, None) == adct.E_SHAPE
    assert f(ctypes.byref(p), 27, 5, None, None, ctypes.byref(p), 0, FAKE, None) == adct.E_SHAPE
    assert f(ctypes.byref(p), 27, 5, None, None, ctypes.byref(p), 32, FAKE + 4, None) == adct.E_ALIGN
    bad = _plane(FAKE, adct.I16, 32, 40, 96)
    assert f(ctypes.byref(bad), 27, 5, None, None, ctypes.byref(bad), 32, None, None) == adct.E_SHAPE


def test_noalloc_scratch_size_matches_header():
    import re
    with open(os.path.join(ROOT, "include", "adct.h")) as f:
        m = re.search(r"#define ADCT_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", f.read())
    assert m, "ADCT_NOALLOC_SCRATCH_BYTES not found"
    assert adct.NOALLOC_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))


def test_t32_constants_and_tables_match_oracle():
    from oracle import t32 as T32
    T, s, W = adct.t32_constants()
    assert np.array_equal(T, T32.transform_matrix_32())
    assert np.array_equal(s, T32.scaling_vector_32())
    assert np.array_equal(W, T32.zonal_weights_32())
    for qp in (0, 4, 22, 27, 37, 51, 63):
        qs, dqs = adct.t32_quant_tables(qp)
        oqs, odqs = T32.quant_tables_32(qp)
        assert np.array_equal(qs.view(np.uint32), oqs.view(np.uint32)), qp
        assert np.array_equal(dqs.view(np.uint32), odqs.view(np.uint32)), qp


def test_t32_kernel_butterflies_count_120_and_match_oracle():
    from oracle import t32 as T32
    A = T32.transform_matrix_32()
    rng = np.random.default_rng(32)
    vecs = list(np.eye(32, dtype=np.int64)) + [rng.integers(-65280, 65281, 32) for _ in range(100)]
    for v in vecs:
        y, n = adct.t32_host_butterfly_count(v)
        assert n == 120 and np.array_equal(y, A @ v)
        x, n = adct.t32_host_butterfly_count(v, inverse=True)
        assert n == 120 and np.array_equal(x, A.T @ v)


def test_t64_constants_and_tables_match_oracle():
    from oracle import t64 as T64
    T, s, W = adct.t64_constants()
    assert np.array_equal(T, T64.transform_matrix_64())
    assert np.array_equal(s, T64.scaling_vector_64())
    assert np.array_equal(W, T64.zonal_weights_64())
    for qp in (0, 4, 15, 16, 22, 27, 37, 51, 63):
        qs, dqs = adct.t64_quant_tables(qp)
        oqs, odqs = T64.quant_tables_64(qp)
        assert np.array_equal(qs.view(np.uint32), oqs.view(np.uint32)), qp
        assert np.array_equal(dqs.view(np.uint32), odqs.view(np.uint32)), qp


def test_t64_kernel_butterflies_count_304_and_match_oracle():
    from oracle import t64 as T64
    A = T64.transform_matrix_64()
    rng = np.random.default_rng(64)
    vecs = list(np.eye(64, dtype=np.int64)) + [rng.integers(-131008, 131009, 64) for _ in range(100)]
    for v in vecs:
        y, n = adct.t64_host_butterfly_count(v)
        assert n == 304 and np.array_equal(y, A @ v)
        x, n = adct.t64_host_butterfly_count(v, inverse=True)
        assert n == 304 and np.array_equal(x, A.T @ v)


def test_serving_constants_match_header():
    import re
    with open(os.path.join(ROOT, "include", "adct.h")) as f:
        defs = dict(re.findall(r"#define ADCT_(SERVE_[A-Z_]+)\s+(\d+)\s*$", f.read(), re.M))
    for name in ("SERVE_PERSISTENT", "SERVE_PLAIN", "SERVE_DMA_ADAPTIVE", "SERVE_DMA_BY_SIZE"):
        assert int(defs[name]) == getattr(adct, name), name
    assert len(adct.ServerCfg._fields_) == 11 and adct.ServerCfg._fields_[-1][0] == "dma_policy"
    assert adct.Stats._fields_[-1][0] == "dma_copies"
