// Grid kernels of the plain and fused entry points (one launch per call,
// TPW tiles per workgroup, one workgroup per tile group).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct_tile.hpp"

namespace adct {

enum FwdOut { kOutCoef = 0, kOutQuant = 1 };
enum InvIn { kInZfix = 0, kInZonal = 1, kInDequant = 2 };
enum InvOut { kOutPlane = 0, kOutBlock = 1 };

struct FwdArgs {
    PlaneRef src;
    uint32_t nblk;
    void* out;   // int32 [nblk][256] (kOutCoef) or int16 (kOutQuant)
    Scale5 qs;   // quantiser scale per class (kOutQuant)
};

struct InvArgs {
    const void* in;     // int32 coef / zfix, or int16 levels
    uint32_t nblk;
    int32_t r;          // zonal size (kInZonal)
    Scale5 dqs;         // dequantiser scale per class (kInDequant)
    PlaneRef dst;       // output plane (kOutPlane)
    int32_t* out_block; // output blocks (kOutBlock)
    PlaneRef ref;       // reference plane for the SSE
    uint32_t ipb;       // tile rows per image
    unsigned long long* sse;
};

// Y = T A T^T per tile; stored as int32 coefficients, or quantised to int16.
template <int TPW, typename S, int OUT>
__global__ __launch_bounds__(TPW * 16) void k_fwd(FwdArgs a) {
    __shared__ int32_t lds[TPW * kLdsTileFwd];
    const int tid = threadIdx.x;
    const uint32_t tile0 = blockIdx.x * (uint32_t)TPW;
    {
        const int lt = tid % TPW, i = tid / TPW;
        const uint32_t g = tile0 + (uint32_t)lt;
        const bool ok = g < a.nblk;
        fwd_row_phase<S>(ok ? tile_row_ptr<S>(a.src, g, i) : nullptr, ok, lt, i, lds);
    }
    __syncthreads();
    {
        const int v = tid & 15, lt = tid >> 4;
        const uint32_t g = tile0 + (uint32_t)lt;
        int32_t y[16];
        fwd_column_phase(lds, lt, v, y);
        if (g < a.nblk) {
            if constexpr (OUT == kOutCoef) {
                int32_t* o = static_cast<int32_t*>(a.out) + (int64_t)g * 256 + v;
#pragma unroll
                for (int u = 0; u < 16; ++u) o[u * 16] = y[u];
            } else {
                float f[3];
                column_factors(a.qs, v, f);
                int16_t* o = static_cast<int16_t*>(a.out) + (int64_t)g * 256 + v;
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int32_t q = round_away(__fmul_rn((float)y[u], f[log2_norm(u) - 2]));
                    o[u * 16] = (int16_t)clamp_i32(q, -32768, 32767);
                }
            }
        }
    }
}

// Fixed-point coefficient column v of tile g, per input mode.
template <int IN>
__device__ __forceinline__ void load_fixed_column(const InvArgs& a, uint32_t g, int v, int32_t (&z)[16]) {
    if constexpr (IN == kInZfix) {
        const int32_t* p = static_cast<const int32_t*>(a.in) + (int64_t)g * 256 + v;
#pragma unroll
        for (int u = 0; u < 16; ++u) z[u] = p[u * 16];
    } else if constexpr (IN == kInZonal) {
        const int32_t* p = static_cast<const int32_t*>(a.in) + (int64_t)g * 256 + v;
        const int lv = log2_norm(v);
        const bool col = v < a.r;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            // W_uv = 256 / (d_u d_v) = 2^(8 - log2 d_u - log2 d_v)
            const int sh = 8 - log2_norm(u) - lv;
            z[u] = (col && u < a.r) ? (int32_t)((uint32_t)p[u * 16] << sh) : 0;
        }
    } else {
        const int16_t* p = static_cast<const int16_t*>(a.in) + (int64_t)g * 256 + v;
        float f[3];
        column_factors(a.dqs, v, f);
#pragma unroll
        for (int u = 0; u < 16; ++u) z[u] = round_away(__fmul_rn((float)p[u * 16], f[log2_norm(u) - 2]));
    }
}

// R = T^T Z' T per tile; stored as int32 blocks, or rounded/clamped into a
// plane with an optional per-image SSE against a reference plane.
template <int TPW, typename S, int IN, int OUT, bool SSE>
__global__ __launch_bounds__(TPW * 16) void k_inv(InvArgs a) {
    __shared__ int32_t lds[TPW * kLdsTileInv];
    const int tid = threadIdx.x;
    const uint32_t tile0 = blockIdx.x * (uint32_t)TPW;
    {
        const int v = tid & 15, lt = tid >> 4;
        const uint32_t g = tile0 + (uint32_t)lt;
        int32_t z[16];
        if (g < a.nblk) {
            load_fixed_column<IN>(a, g, v, z);
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u) z[u] = 0;
        }
        inv_column_phase(z, lt, v, lds);
    }
    __syncthreads();
    if constexpr (OUT == kOutBlock) {
        const int i = tid & 15, lt = tid >> 4;
        const uint32_t g = tile0 + (uint32_t)lt;
        int32_t r[16];
        inv_row_phase(lds, lt, i, r);
        if (g < a.nblk) {
            int4* o = reinterpret_cast<int4*>(a.out_block + (int64_t)g * 256 + i * 16);
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = make_int4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
        }
    } else {
        const int lt = tid % TPW, i = tid / TPW;
        const uint32_t g = tile0 + (uint32_t)lt;
        const bool ok = g < a.nblk;
        int32_t r[16];
        inv_row_phase(lds, lt, i, r);
        round_clamp_row<S>(r);
        int32_t s = 0;
        if (ok) {
            Samples<S>::store(const_cast<char*>(tile_row_ptr<S>(a.dst, g, i)), r);
            if constexpr (SSE) s = row_sse<S>(r, tile_row_ptr<S>(a.ref, g, i));
        }
        if constexpr (SSE) {
            const uint32_t last = min(tile0 + (uint32_t)TPW, a.nblk) - 1u;
            const uint32_t img0 = (tile0 / a.dst.bw) / a.ipb;
            const uint32_t img1 = (last / a.dst.bw) / a.ipb;
            if (img0 == img1) {
                __shared__ int32_t red[TPW * 16 / 64];
                s = wave_sum(s);
                if ((tid & 63) == 0) red[tid >> 6] = s;
                __syncthreads();
                if (tid == 0) {
                    long long t = 0;
#pragma unroll
                    for (int w = 0; w < TPW * 16 / 64; ++w) t += red[w];
                    atomicAdd(a.sse + img0, (unsigned long long)t);
                }
            } else if (ok && s != 0) {
                atomicAdd(a.sse + (g / a.dst.bw) / a.ipb, (unsigned long long)s);
            }
        }
    }
}

// ---- element-wise coefficient-domain kernels (4 coefficients per thread) ---
// Element e = 4t of the [nblk][16][16] array: u = (e >> 4) & 15, v = e & 15.
__device__ __forceinline__ void elem_uv(uint64_t t, int& u, int& v0) {
    u = (int)((t >> 2) & 15u);
    v0 = (int)(t & 3u) * 4;
}

__global__ __launch_bounds__(256) void k_scale(const int4* __restrict__ in, float4* __restrict__ out,
                                               uint64_t n4, Scale5 ss) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n4; t += (uint64_t)gridDim.x * 256ull) {
        int u, v0;
        elem_uv(t, u, v0);
        const int lu = log2_norm(u) - 4;
        const int4 y = in[t];
        float4 o;
        o.x = __fmul_rn((float)y.x, pick5(ss, lu + log2_norm(v0 + 0)));
        o.y = __fmul_rn((float)y.y, pick5(ss, lu + log2_norm(v0 + 1)));
        o.z = __fmul_rn((float)y.z, pick5(ss, lu + log2_norm(v0 + 2)));
        o.w = __fmul_rn((float)y.w, pick5(ss, lu + log2_norm(v0 + 3)));
        out[t] = o;
    }
}

__device__ __forceinline__ int16_t quant1(int32_t y, float f) {
    return (int16_t)clamp_i32(round_away(__fmul_rn((float)y, f)), -32768, 32767);
}

__global__ __launch_bounds__(256) void k_quant(const int4* __restrict__ in, short4* __restrict__ out,
                                               uint64_t n4, Scale5 qs) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n4; t += (uint64_t)gridDim.x * 256ull) {
        int u, v0;
        elem_uv(t, u, v0);
        const int lu = log2_norm(u) - 4;
        const int4 y = in[t];
        short4 o;
        o.x = quant1(y.x, pick5(qs, lu + log2_norm(v0 + 0)));
        o.y = quant1(y.y, pick5(qs, lu + log2_norm(v0 + 1)));
        o.z = quant1(y.z, pick5(qs, lu + log2_norm(v0 + 2)));
        o.w = quant1(y.w, pick5(qs, lu + log2_norm(v0 + 3)));
        out[t] = o;
    }
}

__global__ __launch_bounds__(256) void k_dequant(const short4* __restrict__ in, int4* __restrict__ out,
                                                 uint64_t n4, Scale5 dqs) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n4; t += (uint64_t)gridDim.x * 256ull) {
        int u, v0;
        elem_uv(t, u, v0);
        const int lu = log2_norm(u) - 4;
        const short4 q = in[t];
        int4 o;
        o.x = round_away(__fmul_rn((float)q.x, pick5(dqs, lu + log2_norm(v0 + 0))));
        o.y = round_away(__fmul_rn((float)q.y, pick5(dqs, lu + log2_norm(v0 + 1))));
        o.z = round_away(__fmul_rn((float)q.z, pick5(dqs, lu + log2_norm(v0 + 2))));
        o.w = round_away(__fmul_rn((float)q.w, pick5(dqs, lu + log2_norm(v0 + 3))));
        out[t] = o;
    }
}

__global__ __launch_bounds__(256) void k_zonal(const int4* __restrict__ in, int4* __restrict__ out,
                                               uint64_t n4, int r) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n4; t += (uint64_t)gridDim.x * 256ull) {
        int u, v0;
        elem_uv(t, u, v0);
        const int su = 8 - log2_norm(u);
        const bool row = u < r;
        const int4 y = in[t];
        int4 o;
        o.x = (row && v0 + 0 < r) ? (int32_t)((uint32_t)y.x << (su - log2_norm(v0 + 0))) : 0;
        o.y = (row && v0 + 1 < r) ? (int32_t)((uint32_t)y.y << (su - log2_norm(v0 + 1))) : 0;
        o.z = (row && v0 + 2 < r) ? (int32_t)((uint32_t)y.z << (su - log2_norm(v0 + 2))) : 0;
        o.w = (row && v0 + 3 < r) ? (int32_t)((uint32_t)y.w << (su - log2_norm(v0 + 3))) : 0;
        out[t] = o;
    }
}

// Per-image SSE of two planes; one thread per 16-sample row segment.
template <typename S>
__global__ __launch_bounds__(256) void k_sse(PlaneRef a, PlaneRef b, uint32_t nseg, uint32_t segs_per_row,
                                             uint32_t rows_per_image, unsigned long long* sse) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    int32_t s = 0;
    uint32_t img = 0;
    if (t < nseg) {
        const uint32_t row = t / segs_per_row, seg = t - row * segs_per_row;
        const int64_t off_a = (int64_t)row * a.pitch + (int64_t)seg * 16 * (int64_t)sizeof(S);
        const int64_t off_b = (int64_t)row * b.pitch + (int64_t)seg * 16 * (int64_t)sizeof(S);
        int32_t x[16];
        Samples<S>::load(a.data + off_a, x);
        s = row_sse<S>(x, b.data + off_b);
        img = row / rows_per_image;
    }
    // a workgroup spans at most two images when rows_per_image * segs_per_row >= 256
    const uint32_t t0 = blockIdx.x * 256u;
    const uint32_t tl = min(t0 + 255u, nseg - 1u);
    const uint32_t img0 = (t0 / segs_per_row) / rows_per_image;
    const uint32_t img1 = (tl / segs_per_row) / rows_per_image;
    if (img0 == img1) {
        __shared__ int32_t red[4];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            const long long tot = (long long)red[0] + red[1] + red[2] + red[3];
            atomicAdd(sse + img0, (unsigned long long)tot);
        }
    } else if (t < nseg && s != 0) {
        atomicAdd(sse + img, (unsigned long long)s);
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long* p, uint32_t n) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

}  // namespace adct
