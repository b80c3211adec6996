// Mixed 8/16-point coding: the codec of the paper's second video scenario
// (Section 3.2), in which both the 8-point (T8) and the 16-point (T)
// transforms are the approximations.  Every 16x16 region is coded twice at
// the same QP, as one 16x16 block with T and as four 8x8 blocks with T8, and
// keeps the coding of lower cost J = D + lambda R: D the region's exact sum of
// squared reconstruction errors, R its number of nonzero levels (ties keep
// the 16x16 coding).  Each coding is the plain codec of its size: levels
// q = rnd(fp32(Y) qs), fixed-point coefficients rnd(fp32(q) dqs) with 8 (T)
// or 6 (T8) fractional bits, the integer inverse, and the rounding
// floor((R + half) / 2^bits) clamped to the sample range.
//
// Layout: 16 lanes per region, lane i owning row i of the region's samples;
// a wave codes four consecutive regions per step and runs through a
// contiguous range of regions.  Row passes run in registers; the transposes
// to column passes and back go through a 16 x 17 word LDS array per region
// (conflict-free: lane (g, i) of region slot g touches bank 16 g + 17 i + c
// for row-wise and 16 g + i + 17 r for column-wise access).  The 8x8 coding
// uses the same data movement with T8 on each half row and half column,
// which is the transform of the four 8x8 blocks.  The chosen levels pass
// through LDS once more so that each lane stores one row (32 bytes) of the
// region's block-major level array.
#include <hip/hip_runtime.h>

#include "adct_internal.hpp"
#include "adct_t8_common.hpp"
#include "adct_tile.hpp"

namespace adct {
namespace {

constexpr int kLd = 17;                // LDS row stride (32-bit words)
constexpr int kRegion = 16 * kLd;      // words per region slot
constexpr uint32_t kMaxWaves = 8192;   // waves of a launch (32 per CU)
constexpr uint32_t kNoImage = 0xffffffffu;

struct MixArgs {
    const char* src;
    int64_t src_pitch;
    char* dst;
    int64_t dst_pitch;
    int16_t* q;                  // block-major levels, or null
    uint8_t* split;              // per region, or null
    unsigned long long* sse;     // per image, or null
    uint32_t nreg, bw, per_wave; // regions, regions per block row, regions per wave (multiple of 4)
    FastDiv bwdiv, ipbdiv;       // / bw, / block rows per image
    long long lambda;
    float qs16[5], dqs16[5];     // class log2 d_u + log2 d_v - 4 of T
    float qs8[5], dqs8[5];       // class log2 d_u + log2 d_v - 2 of T8
};

__device__ __forceinline__ void wave_sync() {
    // LDS written by some lanes of the wave, read by others
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float pick(const float (&t)[5], int c) {
    float r = t[4];
    r = (c == 3) ? t[3] : r;
    r = (c == 2) ? t[2] : r;
    r = (c == 1) ? t[1] : r;
    r = (c == 0) ? t[0] : r;
    return r;
}

__device__ __forceinline__ void put_row(int32_t* t, int i, const int32_t (&v)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) t[i * kLd + k] = v[k];
}
__device__ __forceinline__ void get_row(const int32_t* t, int i, int32_t (&v)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[i * kLd + k];
}
__device__ __forceinline__ void put_col(int32_t* t, int j, const int32_t (&v)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) t[r * kLd + j] = v[r];
}
__device__ __forceinline__ void get_col(const int32_t* t, int j, int32_t (&v)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = t[r * kLd + j];
}

// The 1D transform of one coding on a row or column of 16 values: T, or T8
// on each half.
template <bool EIGHT>
__device__ __forceinline__ void fwd_line(const int32_t (&x)[16], int32_t (&y)[16]) {
    if constexpr (EIGHT) {
        int32_t a[8], b[8], ya[8], yb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = x[k];
            b[k] = x[8 + k];
        }
        fwd8(a, ya);
        fwd8(b, yb);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            y[k] = ya[k];
            y[8 + k] = yb[k];
        }
    } else {
        fwd16(x, y);
    }
}

template <bool EIGHT>
__device__ __forceinline__ void inv_line(const int32_t (&y)[16], int32_t (&x)[16]) {
    if constexpr (EIGHT) {
        int32_t a[8], b[8], xa[8], xb[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = y[k];
            b[k] = y[8 + k];
        }
        inv8(a, xa);
        inv8(b, xb);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = xa[k];
            x[8 + k] = xb[k];
        }
    } else {
        inv16(y, x);
    }
}

// log2 d_u - (2 for T, 1 for T8): the index into a lane's three factors
template <bool EIGHT>
__host__ __device__ constexpr int row_class(int u) {
    return EIGHT ? l8(u & 7) - 1 : log2_norm(u) - 2;
}

struct Coded {
    uint32_t q[8];    // levels of the lane's column, pairs (u = 2m, 2m + 1)
    uint32_t out[8];  // reconstruction of the lane's row, pairs (j = 2m, 2m + 1)
    int32_t d, r;     // the lane's share of D (its row) and R (its column)
};

typedef short s16x2 __attribute__((ext_vector_type(2)));

// One coding of the wave's four regions.  Lane (g, i): x is row i of region
// slot g (xw the same samples as 16-bit pairs); on return the lane holds
// column i's levels, row i's reconstruction and its shares of D and R.  fq /
// fd are the lane's quantiser / dequantiser factors for column i, indexed by
// row_class(u).
// SAT: saturate the levels to int16.  Only the 16-point coding of int16
// samples below QP 4 can need it; the 8-point levels stay within
// 8 * 2047 / Delta < 26000 (sqrt(d_u d_v) <= 8 for T8).
template <typename S, bool EIGHT, bool SAT>
__device__ __forceinline__ void code(const int32_t (&x)[16], const uint32_t (&xw)[8], int32_t* t, int i,
                                     const float (&fq)[3], const float (&fd)[3], Coded& c) {
    constexpr int kBits = EIGHT ? 6 : 8;
    int32_t a[16], b[16];
    fwd_line<EIGHT>(x, a);  // row pass
    wave_sync();            // earlier readers of t are done
    put_row(t, i, a);
    wave_sync();
    get_col(t, i, a);
    fwd_line<EIGHT>(a, b);  // column pass: b[u] = Y[u][i]
    c.r = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float v = __fmul_rn((float)b[u], fq[row_class<EIGHT>(u)]);
        const float h = copysignf(0x1.fffffep-2f, v);
        int32_t q = round_away_h(v, h);
        if constexpr (SAT) q = clamp_i32(q, -32768, 32767);
        c.r += q != 0;
        b[u] = round_away_h(__fmul_rn((float)q, fd[row_class<EIGHT>(u)]), h);
        if (u & 1)
            c.q[u >> 1] |= (uint32_t)q << 16;
        else
            c.q[u >> 1] = (uint32_t)q & 0xffffu;
    }
    // rounding offset on each block's DC, which reaches every sample of its
    // block with weight 1
    if constexpr (EIGHT) {
        if ((i & 7) == 0) {
            b[0] += 1 << (kBits - 1);
            b[8] += 1 << (kBits - 1);
        }
    } else {
        if (i == 0) b[0] += 1 << (kBits - 1);
    }
    inv_line<EIGHT>(b, a);  // inverse column pass: a[r] = R1[r][i]
    wave_sync();
    put_col(t, i, a);
    wave_sync();
    get_row(t, i, a);
    inv_line<EIGHT>(a, b);  // inverse row pass: b[j] = R[i][j]
    constexpr int32_t lo = Samples<S>::kLo, hi = Samples<S>::kHi;
    c.d = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        // clamp before the shift: floor((R + half) / 2^bits) lands in [lo, hi]
        const int32_t r0 = clamp_i32(b[2 * m], lo * (1 << kBits), hi * (1 << kBits) + (1 << kBits) - 1);
        const int32_t r1 = clamp_i32(b[2 * m + 1], lo * (1 << kBits), hi * (1 << kBits) + (1 << kBits) - 1);
        uint32_t w;
        if constexpr (kBits == 8)
            w = __builtin_amdgcn_perm((uint32_t)r1, (uint32_t)r0, 0x06050201u);  // bytes 1-2 of each: R >> 8
        else
            w = ((uint32_t)(r0 >> kBits) & 0xffffu) | ((uint32_t)(r1 >> kBits) << 16);
        c.out[m] = w;
        // the two errors as 16-bit lanes, squared and summed by one dot product
        const s16x2 e = __builtin_bit_cast(s16x2, w) - __builtin_bit_cast(s16x2, xw[m]);
        c.d = __builtin_amdgcn_sdot2(e, e, c.d, false);
    }
}

// Sum over the 16 lanes of a region.
__device__ __forceinline__ int32_t region_sum(int32_t v) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename S, bool SSE, bool SAT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_mixed(MixArgs a) {
    __shared__ int32_t lds[4][4 * kRegion];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    int32_t* t = lds[wave] + g * kRegion;
    const uint32_t w = blockIdx.x * 4u + (uint32_t)wave;
    const uint32_t first = w * a.per_wave;
    if (first >= a.nreg) return;
    const uint32_t end = min(a.nreg, first + a.per_wave);
    // the lane's column factors: column i of T's coding, column i % 8 of T8's
    float fq16[3], fd16[3], fq8[3], fd8[3];
    {
        const int lv = log2_norm(i), lv8 = l8(i & 7);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            fq16[k] = pick(a.qs16, k + lv - 2);
            fd16[k] = pick(a.dqs16, k + lv - 2);
            fq8[k] = pick(a.qs8, k + lv8 - 1);
            fd8[k] = pick(a.dqs8, k + lv8 - 1);
        }
    }
    long long acc = 0;
    uint32_t cur = kNoImage;
    for (uint32_t base = first; base < end; base += 4) {
        const uint32_t k = base + (uint32_t)g;
        const bool ok = k < end;
        const uint32_t kk = ok ? k : end - 1;
        const uint32_t by = fdiv(kk, a.bwdiv), bx = kk - by * a.bw;
        const int64_t row = (int64_t)(by * 16u + (uint32_t)i);
        int32_t x[16];
        Samples<S>::load(a.src + row * a.src_pitch + (int64_t)bx * 16 * (int64_t)sizeof(S), x);
        uint32_t xw[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) xw[m] = __builtin_amdgcn_perm((uint32_t)x[2 * m + 1], (uint32_t)x[2 * m], 0x05040100u);
        Coded c16, c8;
        code<S, false, SAT>(x, xw, t, i, fq16, fd16, c16);
        code<S, true, false>(x, xw, t, i, fq8, fd8, c8);
        const int32_t d16 = region_sum(c16.d), d8 = region_sum(c8.d);
        const int32_t rr = region_sum(c16.r | (c8.r << 16));
        const long long j16 = (long long)d16 + a.lambda * (long long)(rr & 0xffff);
        const long long j8 = (long long)d8 + a.lambda * (long long)(rr >> 16);
        const bool use8 = j8 < j16;
        const Coded& ch = use8 ? c8 : c16;
        if (ok) {
            int32_t o[16];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                o[2 * m] = (int32_t)(int16_t)(ch.out[m] & 0xffffu);
                o[2 * m + 1] = (int32_t)ch.out[m] >> 16;
            }
            Samples<S>::store(a.dst + row * a.dst_pitch + (int64_t)bx * 16 * (int64_t)sizeof(S), o);
            if (a.split && i == 0) a.split[k] = use8 ? 1 : 0;
        }
        if (a.q) {
            // levels: column i in the lane -> row i of the block-major array
            int32_t v[16];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                v[2 * m] = (int32_t)(int16_t)(ch.q[m] & 0xffffu);
                v[2 * m + 1] = (int32_t)ch.q[m] >> 16;
            }
            wave_sync();
            put_col(t, i, v);
            wave_sync();
            get_row(t, i, v);
            if (ok) {
                uint32_t p[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) p[m] = ((uint32_t)v[2 * m] & 0xffffu) | ((uint32_t)v[2 * m + 1] << 16);
                char* qp = reinterpret_cast<char*>(a.q) + (int64_t)k * 512 + i * 32;
                store16(qp, make_uint4(p[0], p[1], p[2], p[3]));
                store16(qp + 16, make_uint4(p[4], p[5], p[6], p[7]));
            }
        }
        if constexpr (SSE) {
            // the four regions' D in order; a wave's regions run through the
            // images in order, so each image change flushes one sum
            const int32_t dsel = use8 ? d8 : d16;
            const uint32_t img = fdiv(by, a.ipbdiv);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (base + (uint32_t)s >= end) break;
                const uint32_t im = (uint32_t)__shfl((int)img, s * 16, 64);
                const int32_t ds = __shfl(dsel, s * 16, 64);
                if (im != cur) {
                    if (cur != kNoImage && acc && lane == 0) atomicAdd(a.sse + cur, (unsigned long long)acc);
                    cur = im;
                    acc = 0;
                }
                acc += ds;
            }
        }
    }
    if constexpr (SSE) {
        if (cur != kNoImage && acc && lane == 0) atomicAdd(a.sse + cur, (unsigned long long)acc);
    }
}

__global__ __launch_bounds__(256) void k_mixed_zero(unsigned long long* p, uint32_t n) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

int adct_mixed_encode(const adct_plane* src, int qp, int64_t lambda, int16_t* q, uint8_t* split,
                      const adct_plane* dst, int32_t image_height, int64_t* sse, void* stream) {
    int rc = check_plane(src);
    if (rc) return rc;
    if ((rc = check_plane(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (lambda < 0 || lambda > ADCT_MIXED_MAX_LAMBDA) return ADCT_E_ARG;
    if (q && !aligned16(q)) return ADCT_E_ALIGN;
    if (sse && (image_height <= 0 || (image_height & 15) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    Scale5Host qs, dqs;
    MixArgs a{};
    if (!quant_scales(qp, &qs, &dqs) || !quant_scales8(qp, a.qs8, a.dqs8)) return ADCT_E_ARG;
    for (int c = 0; c < 5; ++c) {
        a.qs16[c] = qs.f[c];
        a.dqs16[c] = dqs.f[c];
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    a.dst = static_cast<char*>(dst->data);
    a.dst_pitch = dst->pitch_bytes;
    a.q = q;
    a.split = split;
    a.sse = reinterpret_cast<unsigned long long*>(sse);
    a.nreg = (uint32_t)plane_blocks(src);
    a.bw = (uint32_t)(src->width / 16);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(sse ? (uint32_t)(image_height / 16) : 1u);
    a.lambda = lambda;
    if (sse) {
        const uint32_t nimg = (uint32_t)(src->height / image_height);
        hipLaunchKernelGGL(k_mixed_zero, dim3((nimg + 255) / 256), dim3(256), 0, s, a.sse, nimg);
        if ((rc = launched())) return rc;
    }
    // a contiguous range of regions per wave, four at a time
    const uint32_t steps = (a.nreg + 3) / 4;
    const uint32_t waves = steps < kMaxWaves ? steps : kMaxWaves;
    a.per_wave = 4 * ((steps + waves - 1) / waves);
    const uint32_t nwaves = (a.nreg + a.per_wave - 1) / a.per_wave;
    const dim3 grid((nwaves + 3) / 4);
    // uint8 levels always fit int16; int16 ones unless QP < 4
    if (src->dtype == ADCT_U8) {
        if (sse)
            hipLaunchKernelGGL((k_mixed<uint8_t, true, false>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_mixed<uint8_t, false, false>), grid, dim3(256), 0, s, a);
    } else if (i16_levels_fit(qs)) {
        if (sse)
            hipLaunchKernelGGL((k_mixed<int16_t, true, false>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_mixed<int16_t, false, false>), grid, dim3(256), 0, s, a);
    } else {
        if (sse)
            hipLaunchKernelGGL((k_mixed<int16_t, true, true>), grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_mixed<int16_t, false, true>), grid, dim3(256), 0, s, a);
    }
    return launched();
}

}  // extern "C"
