// Tile-group building blocks for gfx950.
//
// A workgroup of 16 * TPW threads (TPW = tiles per workgroup) processes TPW
// 16x16 tiles at a time.  Every 2D pass (Section 3.1, B = C A C^T and its
// inverse) is two 1D passes with an LDS-staged transpose between them:
//
//   forward   row phase     thread (lt, i) loads sample row i of tile lt
//                           (16 B of uint8 / 32 B of int16, the TPW tiles of
//                           a group side by side, so neighbouring lanes read
//                           neighbouring bytes), runs fwd16 on it and writes
//                           the 16 results down column i of the tile's LDS
//                           block;
//             column phase  thread (lt, v) reads row v of that LDS block
//                           (= column v of the row-pass output), runs fwd16
//                           and owns Y[0..15][v]; stores go out with lanes of
//                           consecutive v adjacent in memory.
//   inverse   column phase  thread (lt, v) loads coefficient column v (again
//                           lanes of consecutive v adjacent), builds the
//                           fixed-point coefficients (zonal weights or
//                           dequantisation), runs inv16 and writes them down
//                           column v of the LDS block;
//             row phase     thread (lt, i) reads row i, runs inv16, rounds
//                           and clamps, and stores one 16-sample row.
//
// LDS blocks are padded (row stride 20 words, tile stride chosen per
// direction) so that the scattered 4-byte writes of a wavefront fall in
// distinct banks and the row reads can use 16-byte ds_read_b128.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct_butterfly.hpp"

namespace adct {

constexpr int kLdsRow = 20;            // words between LDS rows of a tile
constexpr int kLdsTileFwd = 16 * 20 + 4;   // tile stride, forward direction
constexpr int kLdsTileInv = 16 * 20 + 16;  // tile stride, inverse direction

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
        *reinterpret_cast<uint4*>(p) = make_uint4(ws[0], ws[1], ws[2], ws[3]);
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
        reinterpret_cast<uint4*>(p)[0] = make_uint4(ws[0], ws[1], ws[2], ws[3]);
        reinterpret_cast<uint4*>(p)[1] = make_uint4(ws[4], ws[5], ws[6], ws[7]);
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

// round half away from zero of an fp32 value, as an integer
__device__ __forceinline__ int32_t round_away(float x) { return (int32_t)roundf(x); }

__device__ __forceinline__ int32_t clamp_i32(int32_t x, int32_t lo, int32_t hi) {
    return min(max(x, lo), hi);
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

// ---- forward: sample rows -> LDS ------------------------------------------
// Thread (lt, i): row i of tile lt.  `valid` false loads zeros.
template <typename S>
__device__ __forceinline__ void fwd_row_phase(const char* row_ptr, bool valid, int lt, int i,
                                              int32_t* lds) {
    int32_t x[16], z[16];
    if (valid) {
        Samples<S>::load(row_ptr, x);
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = 0;
    }
    fwd16(x, z);
    int32_t* l = lds + lt * kLdsTileFwd + i;
#pragma unroll
    for (int v = 0; v < 16; ++v) l[v * kLdsRow] = z[v];
}

// Thread (lt, v): column v of the row-pass output -> Y[0..15][v].
__device__ __forceinline__ void fwd_column_phase(const int32_t* lds, int lt, int v, int32_t (&y)[16]) {
    const int4* l = reinterpret_cast<const int4*>(lds + lt * kLdsTileFwd + v * kLdsRow);
    int32_t z[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 w = l[k];
        z[4 * k] = w.x;
        z[4 * k + 1] = w.y;
        z[4 * k + 2] = w.z;
        z[4 * k + 3] = w.w;
    }
    fwd16(z, y);
}

// ---- inverse: coefficient columns -> LDS -> sample rows ---------------------
// Thread (lt, v) holds the fixed-point column zc[u] = Z'[u][v]; after this
// call LDS holds Q = T^T Z' (column v written down LDS column v).
__device__ __forceinline__ void inv_column_phase(const int32_t (&zc)[16], int lt, int v, int32_t* lds) {
    int32_t q[16];
    inv16(zc, q);
    int32_t* l = lds + lt * kLdsTileInv + v;
#pragma unroll
    for (int i = 0; i < 16; ++i) l[i * kLdsRow] = q[i];
}

// Thread (lt, i): R[i][0..15] = (row i of Q) T.
__device__ __forceinline__ void inv_row_phase(const int32_t* lds, int lt, int i, int32_t (&r)[16]) {
    const int4* l = reinterpret_cast<const int4*>(lds + lt * kLdsTileInv + i * kLdsRow);
    int32_t q[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 w = l[k];
        q[4 * k] = w.x;
        q[4 * k + 1] = w.y;
        q[4 * k + 2] = w.z;
        q[4 * k + 3] = w.w;
    }
    inv16(q, r);
}

// floor((R + 128) / 256) clamped to the sample range.  The clamp is applied
// before the shift (floor(clamp(x, 256 lo, 256 hi + 255) / 256) equals
// clamp(floor(x / 256), lo, hi)): written as shift-then-clamp, the compiler
// fuses shift, saturation and byte packing into v_ashr_pk_u8_i32, whose
// upper 16 result bits are not cleared before they are OR-ed with the other
// bytes of the row.
template <typename S>
__device__ __forceinline__ void round_clamp_row(int32_t (&r)[16]) {
#pragma unroll
    for (int j = 0; j < 16; ++j)
        r[j] = clamp_i32(r[j] + 128, Samples<S>::kLo * 256, Samples<S>::kHi * 256 + 255) >> 8;
}

// Sum of squared differences of a reconstructed row against a reference row.
template <typename S>
__device__ __forceinline__ int32_t row_sse(const int32_t (&o)[16], const char* ref_row) {
    int32_t x[16];
    Samples<S>::load(ref_row, x);
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int32_t e = o[j] - x[j];
        s += e * e;
    }
    return s;
}

// Wave64 sum.
__device__ __forceinline__ int32_t wave_sum(int32_t s) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    return s;
}

}  // namespace adct
