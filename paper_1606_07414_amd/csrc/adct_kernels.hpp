// Element-wise coefficient-domain kernels, the plane SSE and small fills
// (non-template kernels: include from one translation unit only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct_tile.hpp"

namespace adct {

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

__global__ __launch_bounds__(256) void k_zigzag(const int4* __restrict__ in, int4* __restrict__ out,
                                                uint64_t n4, int r) {
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n4; t += (uint64_t)gridDim.x * 256ull) {
        int u, v0;
        elem_uv(t, u, v0);
        const int su = 8 - log2_norm(u);
        const int4 y = in[t];
        int4 o;
        o.x = zigzag_rank(u, v0 + 0) < r ? (int32_t)((uint32_t)y.x << (su - log2_norm(v0 + 0))) : 0;
        o.y = zigzag_rank(u, v0 + 1) < r ? (int32_t)((uint32_t)y.y << (su - log2_norm(v0 + 1))) : 0;
        o.z = zigzag_rank(u, v0 + 2) < r ? (int32_t)((uint32_t)y.z << (su - log2_norm(v0 + 2))) : 0;
        o.w = zigzag_rank(u, v0 + 3) < r ? (int32_t)((uint32_t)y.w << (su - log2_norm(v0 + 3))) : 0;
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
