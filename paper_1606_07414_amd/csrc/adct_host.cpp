// Host-only parts of the C ABI: constants, quantisation tables, PSNR and the
// host execution of the butterflies.  No HIP calls, so all of it runs
// without a GPU.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "adct.h"
#include "adct_internal.hpp"
#include "adct_t8_common.hpp"
#include "adct_t32_common.hpp"
#include "adct_t64_common.hpp"
#include "adct_round.hpp"

namespace adct {

// T of Section 2.1 (library copy; row u is output frequency u).
static const int8_t kT[16][16] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, 1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1, -1, -1},
    {1, 0, 0, 0, 0, 0, 0, -1, -1, 0, 0, 0, 0, 0, 0, 1},
    {1, 1, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, -1, -1},
    {1, 0, 0, -1, -1, 0, 0, 1, 1, 0, 0, -1, -1, 0, 0, 1},
    {1, 1, -1, -1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1},
    {0, 0, -1, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, -1, 0, 0},
    {0, 0, 0, 0, 0, 0, -1, 1, -1, 1, 0, 0, 0, 0, 0, 0},
    {1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 0, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 0, 0},
    {0, -1, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, -1, 0},
    {0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0},
    {0, -1, 1, 0, 0, 1, -1, 0, 0, -1, 1, 0, 0, 1, -1, 0},
    {1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1},
    {0, 0, 0, -1, 1, 0, 0, 0, 0, 0, 0, 1, -1, 0, 0, 0},
    {0, 0, 0, 0, -1, 1, 0, 0, 0, 0, -1, 1, 0, 0, 0, 0},
};

static int row_norm(int u) {
    int d = 0;
    for (int j = 0; j < 16; ++j) d += kT[u][j] * kT[u][j];
    return d;
}

// s_u s_v for a class c = log2 d_u + log2 d_v - 4: 1 / sqrt(d_u d_v).
static double class_ss(int c) { return 1.0 / sqrt((double)(1 << (c + 4))); }

bool quant_scales(int qp, Scale5Host* qs, Scale5Host* dqs) {
    if (qp < 0 || qp > 63) return false;
    const double delta = exp2((qp - 4) / 6.0);
    for (int c = 0; c < 5; ++c) {
        const double ss = class_ss(c);
        if (qs) qs->f[c] = (float)(ss / delta);
        if (dqs) dqs->f[c] = (float)(256.0 * delta * ss);
    }
    return true;
}

// In class c (d_u d_v = 2^(c+4)) every coefficient has |Y| <= d_u d_v * 2047,
// T's entries being 0 or +-1; a bound below 32767 keeps the fp32 product
// below 32767.5, so its level is at most 32767 in magnitude.  (uint8 planes,
// |Y s_u s_v| <= 4080, always fit.)
bool i16_levels_fit(const Scale5Host& qs) {
    for (int c = 0; c < 5; ++c)
        if ((double)qs.f[c] * 2047.0 * (double)(16 << c) >= 32767.0) return false;
    return true;
}

void ortho_scales(Scale5Host* ss) {
    for (int c = 0; c < 5; ++c) ss->f[c] = (float)class_ss(c);
}

int class_of(int u, int v) {
    int lu = 0, lv = 0;
    for (int d = row_norm(u); d > 1; d >>= 1) ++lu;
    for (int d = row_norm(v); d > 1; d >>= 1) ++lv;
    return lu + lv - 4;
}

// An integer that counts the additions and subtractions made with it.  It
// defines no other arithmetic, so a butterfly instantiated with it compiles
// only if its dataflow is additions and subtractions alone (no negation,
// multiply or shift).
struct CountedInt {
    int64_t v = 0;
    static thread_local int64_t ops;
};
thread_local int64_t CountedInt::ops = 0;
inline CountedInt operator+(CountedInt a, CountedInt b) {
    ++CountedInt::ops;
    return CountedInt{a.v + b.v};
}
inline CountedInt operator-(CountedInt a, CountedInt b) {
    ++CountedInt::ops;
    return CountedInt{a.v - b.v};
}

}  // namespace adct

using namespace adct;

extern "C" {

int adct_abi_version(void) { return ADCT_ABI_VERSION; }

int adct_constants(int32_t* T256, double* s16, int32_t* W256) {
    for (int u = 0; u < 16; ++u) {
        if (T256)
            for (int j = 0; j < 16; ++j) T256[u * 16 + j] = kT[u][j];
        if (s16) s16[u] = 1.0 / sqrt((double)row_norm(u));
        if (W256)
            for (int v = 0; v < 16; ++v) W256[u * 16 + v] = 256 / (row_norm(u) * row_norm(v));
    }
    return ADCT_OK;
}

int adct_round_check(uint32_t first_bits, uint32_t count, int64_t* mismatches) {
    if (!mismatches) return ADCT_E_ARG;
    int64_t bad = 0;
    for (uint64_t k = 0; k < count; ++k) {
        const uint32_t bits = first_bits + (uint32_t)k;
        float x;
        memcpy(&x, &bits, sizeof x);
        const float r = roundf(x);
        if (!(fabsf(r) < 2147483648.0f)) continue;  // NaN, infinity, or outside int32
        if (round_away(x) != (int32_t)r) ++bad;
    }
    *mismatches = bad;
    return ADCT_OK;
}

int adct_zigzag_ranks(int32_t* rank256) {
    if (!rank256) return ADCT_E_ARG;
    for (int u = 0; u < 16; ++u)
        for (int v = 0; v < 16; ++v) rank256[u * 16 + v] = zigzag_rank(u, v);
    return ADCT_OK;
}

int adct_quant_tables(int qp, float* qs256, float* dqs256) {
    Scale5Host q, d;
    if (!quant_scales(qp, &q, &d)) return ADCT_E_ARG;
    for (int u = 0; u < 16; ++u)
        for (int v = 0; v < 16; ++v) {
            const int c = class_of(u, v);
            if (qs256) qs256[u * 16 + v] = q.f[c];
            if (dqs256) dqs256[u * 16 + v] = d.f[c];
        }
    return ADCT_OK;
}

int adct_psnr(const int64_t* sse, int32_t n, double pixels_per_image, double peak, double* out) {
    if (!sse || !out || n < 0 || !(pixels_per_image > 0) || !(peak > 0)) return ADCT_E_ARG;
    for (int32_t i = 0; i < n; ++i) {
        if (sse[i] < 0) return ADCT_E_ARG;
        out[i] = sse[i] == 0 ? INFINITY : 10.0 * log10(peak * peak * pixels_per_image / (double)sse[i]);
    }
    return ADCT_OK;
}

int adct_default_tune(adct_tune* out) {
    if (!out) return ADCT_E_ARG;
    // 32-tile groups, 64-tile items, 4 resident workgroups of 256 threads per
    // CU: the fastest measured shape on uneven and uniform batches alike
    out->tiles_per_group = 32;
    out->groups_per_item = 2;
    out->wgs_per_cu = 4;
    out->reserved = 0;
    return ADCT_OK;
}

// Host execution of the kernels' 1D butterflies (the same code the GPU
// runs), for checking the dataflow without a GPU.
int adct_host_butterfly_count(int32_t which, const int32_t* in16, int32_t* out16, int64_t* additions) {
    if (!in16 || !out16 || !additions || which < 0 || which > 4) return ADCT_E_ARG;
    CountedInt x[16], y[16];
    CountedInt::ops = 0;
    for (int i = 0; i < 16; ++i) x[i].v = in16[i];
    if (which >= 3) {
        for (int h = 0; h < 2; ++h) {
            CountedInt a[8], b[8];
            for (int i = 0; i < 8; ++i) a[i] = x[8 * h + i];
            if (which == 3)
                fwd8(a, b);
            else
                inv8(a, b);
            for (int i = 0; i < 8; ++i) y[8 * h + i] = b[i];
        }
    } else if (which == 2)
        wht16(x, y);
    else if (which == 1)
        inv16(x, y);
    else
        fwd16(x, y);
    for (int i = 0; i < 16; ++i) {
        if (y[i].v < INT32_MIN || y[i].v > INT32_MAX) return ADCT_E_ARG;
        out16[i] = (int32_t)y[i].v;
    }
    *additions = CountedInt::ops;
    return ADCT_OK;
}

int adct_t32_constants(int32_t* T1024, double* s32, int32_t* W1024) {
    // T32 = P32 diag(T, T) B32: row 2k is row k of T on the folded sums
    // (T32[2k][j] = T32[2k][31-j] = T[k][j]), row 2k+1 row k of T on the
    // folded differences (T32[2k+1][j] = -T32[2k+1][31-j] = T[k][j])
    for (int u = 0; u < 32; ++u) {
        const int k = u >> 1, odd = u & 1;
        if (T1024)
            for (int j = 0; j < 16; ++j) {
                T1024[u * 32 + j] = kT[k][j];
                T1024[u * 32 + 31 - j] = odd ? -kT[k][j] : kT[k][j];
            }
        if (s32) s32[u] = 1.0 / sqrt((double)(1 << l32(u)));
        if (W1024)
            for (int v = 0; v < 32; ++v) W1024[u * 32 + v] = 1024 >> (l32(u) + l32(v));
    }
    return ADCT_OK;
}

int adct_t32_quant_tables(int qp, float* qs1024, float* dqs1024) {
    float qs[5], dqs[5];
    if (!quant_scales32(qp, qs, dqs)) return ADCT_E_ARG;
    for (int u = 0; u < 32; ++u)
        for (int v = 0; v < 32; ++v) {
            const int c = l32(u) + l32(v) - 6;
            if (qs1024) qs1024[u * 32 + v] = qs[c];
            if (dqs1024) dqs1024[u * 32 + v] = dqs[c];
        }
    return ADCT_OK;
}

int adct_t32_host_butterfly_count(int32_t which, const int32_t* in32, int32_t* out32, int64_t* additions) {
    if (!in32 || !out32 || !additions || which < 0 || which > 1) return ADCT_E_ARG;
    CountedInt x[32], y[32];
    CountedInt::ops = 0;
    for (int i = 0; i < 32; ++i) x[i].v = in32[i];
    if (which == 0)
        fwd32(x, y);
    else
        inv32(x, y);
    for (int i = 0; i < 32; ++i) {
        if (y[i].v < INT32_MIN || y[i].v > INT32_MAX) return ADCT_E_ARG;
        out32[i] = (int32_t)y[i].v;
    }
    *additions = CountedInt::ops;
    return ADCT_OK;
}

// Entry (u, j) of T32 = P32 diag(T, T) B32.
static int t32_entry(int u, int j) {
    const int k = u >> 1, sgn = (u & 1) ? -1 : 1;
    return j < 16 ? kT[k][j] : sgn * kT[k][31 - j];
}

int adct_t64_constants(int32_t* T4096, double* s64, int32_t* W4096) {
    // T64 = P64 diag(T32, T32) B64: row 2k is row k of T32 on the folded sums
    // (T64[2k][j] = T64[2k][63-j] = T32[k][j]), row 2k+1 row k of T32 on the
    // folded differences (T64[2k+1][j] = -T64[2k+1][63-j] = T32[k][j])
    for (int u = 0; u < 64; ++u) {
        const int k = u >> 1, odd = u & 1;
        if (T4096)
            for (int j = 0; j < 32; ++j) {
                T4096[u * 64 + j] = t32_entry(k, j);
                T4096[u * 64 + 63 - j] = odd ? -t32_entry(k, j) : t32_entry(k, j);
            }
        if (s64) s64[u] = 1.0 / sqrt((double)(1 << l64(u)));
        if (W4096)
            for (int v = 0; v < 64; ++v) W4096[u * 64 + v] = 4096 >> (l64(u) + l64(v));
    }
    return ADCT_OK;
}

int adct_t64_quant_tables(int qp, float* qs4096, float* dqs4096) {
    float qs[5], dqs[5];
    if (!quant_scales64(qp, qs, dqs)) return ADCT_E_ARG;
    for (int u = 0; u < 64; ++u)
        for (int v = 0; v < 64; ++v) {
            const int c = l64(u) + l64(v) - 8;
            if (qs4096) qs4096[u * 64 + v] = qs[c];
            if (dqs4096) dqs4096[u * 64 + v] = dqs[c];
        }
    return ADCT_OK;
}

int adct_t64_host_butterfly_count(int32_t which, const int32_t* in64, int32_t* out64, int64_t* additions) {
    if (!in64 || !out64 || !additions || which < 0 || which > 1) return ADCT_E_ARG;
    CountedInt x[64], y[64];
    CountedInt::ops = 0;
    for (int i = 0; i < 64; ++i) x[i].v = in64[i];
    if (which == 0)
        fwd64(x, y);
    else
        inv64(x, y);
    for (int i = 0; i < 64; ++i) {
        if (y[i].v < INT32_MIN || y[i].v > INT32_MAX) return ADCT_E_ARG;
        out64[i] = (int32_t)y[i].v;
    }
    *additions = CountedInt::ops;
    return ADCT_OK;
}

int adct_host_butterfly(int32_t which, const int32_t* in16, int32_t* out16) {
    if (!in16 || !out16 || which < 0 || which > 4) return ADCT_E_ARG;
    int32_t x[16], y[16];
    memcpy(x, in16, sizeof x);
    if (which >= 3) {
        // T8 or T8^T on each half, as the 8x8 and the mixed codecs apply it
        for (int h = 0; h < 2; ++h) {
            int32_t a[8], b[8];
            memcpy(a, x + 8 * h, sizeof a);
            if (which == 3)
                fwd8(a, b);
            else
                inv8(a, b);
            memcpy(y + 8 * h, b, sizeof b);
        }
    } else if (which == 2)
        wht16(x, y);
    else if (which == 1)
        inv16(x, y);
    else
        fwd16(x, y);
    memcpy(out16, y, sizeof y);
    return ADCT_OK;
}

}  // extern "C"
