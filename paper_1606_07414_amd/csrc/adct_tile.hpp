// Sample rows, per-class scale factors, plane addressing and reductions used
// by the tile kernels.
#pragma once

#include "adct_round.hpp"
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct_butterfly.hpp"

namespace adct {

// 16-byte store of streamed output (written once, not read back by the
// kernel).  Nontemporal by default: measured on MI355X, streaming the
// coefficient and sample outputs past the caches raises the fused encoder
// from about 5.1 to 6.3 TB/s.
__device__ __forceinline__ void store16(void* p, uint4 w) {
#ifndef ADCT_CACHED_STORES
    typedef unsigned v4u __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(v4u, w), static_cast<v4u*>(p));
#else
    *static_cast<uint4*>(p) = w;
#endif
}

// 16-byte store of a row piece of a sample plane written straight from the
// row role, through the cache, for planes whose tile-group row segments
// begin or end inside 128-byte lines (a pitch, base or row length that is
// not a multiple of 128 bytes): the neighbouring group writes the rest of
// such a line, and the cache merges the two parts where nontemporal stores
// leave both partial.  Measured on the uneven 4096-image batch (most widths
// not multiples of 128): 5.13 -> 5.63 TB/s.  Planes of whole lines keep the
// nontemporal stores: there the two forms tie, and cached output would push
// out of the Infinity Cache the inputs that a later call reads again.
__device__ __forceinline__ void store16_rowpiece(void* p, uint4 w) { *static_cast<uint4*>(p) = w; }

// Whether the tile-group row segments of an output plane can begin or end
// inside a 128-byte line: its base, pitch or row length (bytes) is not a
// multiple of 128.  A group is a run of whole tiles in raster order whose
// row segment is a multiple of 128 bytes long, so with all three multiples
// of 128 every segment is whole lines.  Uniform over a launch's plane.
__device__ __forceinline__ bool shares_lines(const void* base, int64_t pitch, uint64_t row_bytes) {
    return (((uintptr_t)base | (uint64_t)pitch | row_bytes) & 127u) != 0;
}

// A 16-byte row piece: through the cache on planes whose segments share
// lines with their neighbours', streamed past it otherwise.
__device__ __forceinline__ void store16_row(void* p, uint4 w, bool shared) {
    if (shared)
        store16_rowpiece(p, w);
    else
        store16(p, w);
}

// ---- sample rows --------------------------------------------------------
template <typename S>
struct Samples;

template <>
struct Samples<uint8_t> {
    static constexpr int kLo = 0, kHi = 255;
    static __device__ __forceinline__ void load(const void* p, int32_t (&x)[16]) {
        const uint4 w = *reinterpret_cast<const uint4*>(p);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int b = 0; b < 4; ++b) x[4 * k + b] = (int32_t)((ws[k] >> (8 * b)) & 0xffu);
        }
    }
    // values already within [kLo, kHi]
    static __device__ __forceinline__ void store(void* p, const int32_t (&x)[16]) {
        uint32_t ws[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            ws[k] = (uint32_t)x[4 * k] | ((uint32_t)x[4 * k + 1] << 8) |
                    ((uint32_t)x[4 * k + 2] << 16) | ((uint32_t)x[4 * k + 3] << 24);
        store16(p, make_uint4(ws[0], ws[1], ws[2], ws[3]));
    }
};

template <>
struct Samples<int16_t> {
    static constexpr int kLo = -255, kHi = 255;
    static __device__ __forceinline__ void load(const void* p, int32_t (&x)[16]) {
        const uint4 w0 = reinterpret_cast<const uint4*>(p)[0];
        const uint4 w1 = reinterpret_cast<const uint4*>(p)[1];
        const uint32_t ws[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[2 * k] = (int32_t)(int16_t)(ws[k] & 0xffffu);
            x[2 * k + 1] = (int32_t)(int16_t)(ws[k] >> 16);
        }
    }
    static __device__ __forceinline__ void store(void* p, const int32_t (&x)[16]) {
        uint32_t ws[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            ws[k] = ((uint32_t)x[2 * k] & 0xffffu) | ((uint32_t)x[2 * k + 1] << 16);
        store16(p, make_uint4(ws[0], ws[1], ws[2], ws[3]));
        store16(static_cast<char*>(p) + 16, make_uint4(ws[4], ws[5], ws[6], ws[7]));
    }
};

// ---- per-coefficient scale factors -------------------------------------
// s_u s_v depends on (u, v) only through c = log2 d_u + log2 d_v - 4 in
// 0..4, so every table (quantiser, dequantiser, orthonormal scale) is five
// numbers.  Five-way selects keep them in registers.
struct Scale5 {
    float f[5];
};

__device__ __forceinline__ float pick5(const Scale5& t, int c) {
    float r = t.f[4];
    r = (c == 3) ? t.f[3] : r;
    r = (c == 2) ? t.f[2] : r;
    r = (c == 1) ? t.f[1] : r;
    r = (c == 0) ? t.f[0] : r;
    return r;
}

// Per-thread factors for a fixed column v: out[l - 2] = t[l + log2 d_v - 4]
// for the three possible log2 d_u = l in {2, 3, 4}.
__device__ __forceinline__ void column_factors(const Scale5& t, int v, float (&out)[3]) {
    const int lv = log2_norm(v);
#pragma unroll
    for (int l = 2; l <= 4; ++l) out[l - 2] = pick5(t, l + lv - 4);
}



__device__ __forceinline__ int32_t clamp_i32(int32_t x, int32_t lo, int32_t hi) {
    return min(max(x, lo), hi);
}

// ---- division by a run-time invariant ------------------------------------
// n / d for 32-bit n with a multiplier prepared on the host (round-up
// method of Granlund and Montgomery): l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, q = (t + ((n - t) >> min(l,1))) >> max(l-1,0)
// with t = mulhi(n, m).  Exact for every n < 2^32 and d >= 1.
struct FastDiv {
    uint32_t m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    FastDiv f;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 0 ? l - 1 : 0;
    return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t t = __umulhi(n, f.m);
#else
    const uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// ---- where a tile lives ------------------------------------------------
// A run of tiles inside one plane: tile index g (raster order within the
// plane) -> sample address.
struct PlaneRef {
    const char* data;
    int64_t pitch;   // bytes
    uint32_t bw;     // tiles per row (width / 16)
};

template <typename S>
__device__ __forceinline__ const char* tile_row_ptr(const PlaneRef& p, uint32_t g, int row) {
    const uint32_t by = g / p.bw;
    const uint32_t bx = g - by * p.bw;
    return p.data + (int64_t)(by * 16u + (uint32_t)row) * p.pitch + (int64_t)bx * 16 * (int64_t)sizeof(S);
}

// Sum of squared differences of 16 output samples against a reference row
// held as raw words (uint8: 16 bytes in w0; int16: 8 samples each in w0, w1).
template <typename S>
__device__ __forceinline__ int32_t row_sse_words(const int32_t (&o)[16], uint4 w0, uint4 w1) {
    const uint32_t a[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        int32_t x;
        if constexpr (sizeof(S) == 1)
            x = (int32_t)((a[j >> 2] >> (8 * (j & 3))) & 0xffu);
        else
            x = (j & 1) ? ((int32_t)a[j >> 1] >> 16) : (int32_t)(int16_t)(a[j >> 1] & 0xffffu);
        const int32_t e = o[j] - x;
        s += e * e;
    }
    return s;
}

// Exact SSE of a 16-sample row segment of two planes.
template <typename S>
__device__ __forceinline__ int32_t row_sse(const int32_t (&o)[16], const char* ref_row) {
    const uint4 w0 = reinterpret_cast<const uint4*>(ref_row)[0];
    const uint4 w1 = sizeof(S) == 2 ? reinterpret_cast<const uint4*>(ref_row)[1] : make_uint4(0, 0, 0, 0);
    return row_sse_words<S>(o, w0, w1);
}

// Wave64 sum.
__device__ __forceinline__ int32_t wave_sum(int32_t s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

}  // namespace adct
