// The tile-group processor: every device entry point is one configuration
// of `process_group`, either run over a short chunk of groups per workgroup
// (plain calls: one group, or two where that pays, see kSseGpw and
// kZoneGpw) or called in a loop by a persistent workgroup (batches,
// serving).
//
// A group is TPW tiles of one plane, consecutive in raster order.  It is
// processed by 8 * TPW threads; each thread owns two sample rows (i, i+8) of
// one tile in the "row role" and two coefficient columns (p, p+8) of one
// tile in the "column role":
//
//   row role     lt = tid % TPW, ip = tid / TPW   (lanes of consecutive lt
//                read/write horizontally adjacent 16-sample segments)
//   column role  lt = tid / 8,   p  = tid % 8     (lanes of consecutive p
//                touch adjacent coefficients)
//
// Forward (Section 3.1, Y = T A T^T, each 1D pass the Section 2.2 dataflow):
//   row pass     the two rows are packed as 16-bit pairs and transformed
//                together with packed 16-bit add/sub (one instruction = two
//                rows); results go to LDS as (column p, column p+8) pairs;
//   column pass  the two columns are again one packed pair.  For uint8
//                input every forward quantity is exact modulo 2^16: DC lies
//                in [0, 65280] and every other coefficient in
//                [-32640, 32640], so the 16-bit results are widened by zero
//                extension (DC) or sign extension (the rest).  int16
//                residuals (|Y| up to 65280 anywhere) widen after the row
//                pass and run the column pass in int32.
// Coefficient domain (registers, columns p and p+8): int32 coefficients,
//   quantisation with S folded into the step (Section 2.1), dequantisation to
//   8 fractional bits, or zonal retention with W = 256/(d_u d_v).
// Inverse (Section 3.1, T^T Z' T): column pass in int32, LDS transpose, row
//   pass, rounding floor((R + 128) / 256) and clamping.  The +128 is added
//   once per tile to Z'[0][0]: T^T e0 e0^T T is the all-ones matrix, so it
//   reaches every sample.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct_butterfly.hpp"
#include "adct_tile.hpp"

namespace adct {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u16x2 as_u16x2(uint32_t w) { return __builtin_bit_cast(u16x2, w); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ int32_t sext_lo(uint32_t w) { return (int32_t)(int16_t)(w & 0xffffu); }
__device__ __forceinline__ int32_t sext_hi(uint32_t w) { return (int32_t)w >> 16; }
__device__ __forceinline__ uint32_t perm(uint32_t hi_src, uint32_t lo_src, uint32_t sel) {
    return __builtin_amdgcn_perm(hi_src, lo_src, sel);
}

// LDS geometry (32-bit words).  Forward pairs: [tile][row k][pair p], 8
// words per row; int32 blocks: [tile][row][col], 16 words per row.  Both
// tile strides are 8 (mod 32) so that the lanes of a column-role access hit
// distinct banks.
constexpr int kPairTile = 16 * 8 + 8;   // 136
constexpr int kIntRow = 16;
constexpr int kIntTile = 16 * 16 + 8;   // 264
constexpr int lds_words(int tpw) { return tpw * kIntTile; }

enum InKind { kInSamples = 0, kInY = 1, kInZfix = 2, kInQ = 3 };
enum CStore { kStoreNone = 0, kStoreY = 1, kStoreQ = 2 };
// kMidQuantFit quantises like kMidQuant for inputs whose levels are known
// to fit int16, without the saturation.
enum Mid { kMidNone = 0, kMidZonal = 1, kMidQuant = 2, kMidDequant = 3, kMidZigzag = 4, kMidQuantFit = 5 };
enum OutKind { kOutNothing = 0, kOutSamples = 1, kOutBlocks = 2 };

// XF selects the transform: kXfProposed (T) or kXfWht (comparison).
template <int IN_, int STORE_, int MID_, int OUT_, int ZR_, bool SSE_, int XF_ = kXfProposed>
struct Mode {
    static constexpr int IN = IN_, STORE = STORE_, MID = MID_, OUT = OUT_, ZR = ZR_, XF = XF_;
    static constexpr bool SSE = SSE_;
};

// One group's location and the call's parameters.
struct GroupArgs {
    PlaneRef src;            // samples in (kInSamples)
    PlaneRef dst;            // samples out (kOutSamples)
    PlaneRef ref;            // SSE reference when samples are not the input
    const void* cin;         // coefficient-domain input, block-major
    void* cout;              // int32 Y or int16 q out, block-major
    int32_t* bout;           // int32 blocks out (kOutBlocks)
    int32_t r;               // zonal size when not fixed at compile time
    Scale5 qs, dqs;          // quantiser / dequantiser per class
    uint32_t bw;             // tiles per row of every plane of the call
    FastDiv bwdiv;           // division by bw
    FastDiv ipbdiv;          // division by tile rows per image (SSE image index)
    unsigned long long* sse; // per-image SSE accumulators
    uint32_t image_tiles;    // tiles per image (launch geometry only)
};

// A device address as a pointer the compiler knows to be in global memory.
// Pointers read from memory (a job table, rather than kernel arguments) are
// generic to it, and it would access them with flat instructions; flat
// memory operations also count against the counter that LDS and scalar
// loads wait on, so every wait of an LDS transpose would then wait for the
// outstanding HBM traffic as well.
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
    typedef __attribute__((address_space(1))) T gT;
    return (T*)(gT*)(uintptr_t)p;
}

// GroupArgs read from memory, with every pointer marked global.
__device__ __forceinline__ GroupArgs global_args(GroupArgs a) {
    a.src.data = as_global(a.src.data);
    a.dst.data = as_global(a.dst.data);
    a.ref.data = as_global(a.ref.data);
    a.cin = as_global(a.cin);
    a.cout = as_global(a.cout);
    a.bout = as_global(a.bout);
    a.sse = as_global(a.sse);
    return a;
}

// ---- sample rows as 16-bit pairs ------------------------------------------------
// Rows ip and ip+8 of a tile, raw words (uint8: 16 samples in a0; int16: 8
// samples each in a0, a1; likewise b for row ip+8), as 16 packed pairs
// (row ip sample k, row ip+8 sample k): uint8 zero-extended, int16 as is.
template <typename S>
__device__ __forceinline__ void pack_rows(uint4 a0, uint4 a1, uint4 b0, uint4 b1, uint32_t (&xk)[16]) {
    if constexpr (sizeof(S) == 1) {
        const uint32_t a[4] = {a0.x, a0.y, a0.z, a0.w}, b[4] = {b0.x, b0.y, b0.z, b0.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t m = (uint32_t)(k & 3);
            xk[k] = perm(b[k >> 2], a[k >> 2], 0x0c000c00u | ((4u + m) << 16) | m);
        }
    } else {
        const uint32_t a[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const uint32_t b[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) xk[k] = perm(b[k >> 1], a[k >> 1], (k & 1) ? 0x07060302u : 0x05040100u);
    }
}

// Address of sample row `row` of the tile at tile-row by, tile-column bx.
template <typename S>
__device__ __forceinline__ const char* row_ptr(const PlaneRef& pl, uint32_t by, uint32_t bx, int row) {
    return pl.data + (int64_t)(by * 16u + (uint32_t)row) * pl.pitch + (int64_t)bx * (16 * (int64_t)sizeof(S));
}

// Loads rows ip and ip+8 of tile (by, bx) (zeros when !ok) as raw words.
template <typename S>
__device__ __forceinline__ void load_rows(const PlaneRef& pl, uint32_t by, uint32_t bx, bool ok, int ip, uint4& a0,
                                          uint4& a1, uint4& b0, uint4& b1) {
    a0 = a1 = b0 = b1 = make_uint4(0, 0, 0, 0);
    if (ok) {
        const char* pa = row_ptr<S>(pl, by, bx, ip);
        const char* pb = pa + 8 * pl.pitch;
        a0 = reinterpret_cast<const uint4*>(pa)[0];
        b0 = reinterpret_cast<const uint4*>(pb)[0];
        if constexpr (sizeof(S) == 2) {
            a1 = reinterpret_cast<const uint4*>(pa)[1];
            b1 = reinterpret_cast<const uint4*>(pb)[1];
        }
    }
}

// Exact SSE of the two output rows r0, r1 (clamped 8-fraction-bit values,
// whose samples are byte 1 (uint8) or bytes 1-2 (int16)) against packed
// input pairs: 16-bit differences, squared and accumulated two at a time by
// v_dot2_i32_i16.
template <typename S>
__device__ __forceinline__ int32_t pair_sse(const int32_t (&r0)[16], const int32_t (&r1)[16],
                                            const uint32_t (&xk)[16]) {
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t o = sizeof(S) == 1 ? perm((uint32_t)r1[j], (uint32_t)r0[j], 0x0c050c01u)
                                          : perm((uint32_t)r1[j], (uint32_t)r0[j], 0x06050201u);
        const s16x2 d = __builtin_bit_cast(s16x2, o) - __builtin_bit_cast(s16x2, xk[j]);
        s = __builtin_amdgcn_sdot2(d, d, s, false);
    }
    return s;
}

// ---- forward row pass (row role) -------------------------------------------
// Loads rows ip and ip+8 of tile g and leaves the packed row-pass output in
// LDS pairs.  `xk` keeps the packed input samples for the SSE.
// Raw sample words of rows ip and ip+8 of one tile (row role).
struct RowWords {
    uint4 a0, a1, b0, b1;
    uint4 z[8];  // zone words of a zonal reconstruction (prefetch_zone)
};

template <typename S, int XF>
__device__ __forceinline__ void fwd_rows(const RowWords& w, int lt, int ip, uint32_t* lds, uint32_t (&xk)[16]) {
    pack_rows<S>(w.a0, w.a1, w.b0, w.b1, xk);
    u16x2 x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = as_u16x2(xk[k]);
    u16x2 z[16];
    xf_fwd<XF>(x, z);
    uint32_t w0[8], w1[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        w0[p] = perm(as_u32(z[p + 8]), as_u32(z[p]), 0x05040100u);  // row ip:   (Z[ip][p], Z[ip][p+8])
        w1[p] = perm(as_u32(z[p + 8]), as_u32(z[p]), 0x07060302u);  // row ip+8
    }
    uint4* l0 = reinterpret_cast<uint4*>(lds + lt * kPairTile + ip * 8);
    uint4* l1 = reinterpret_cast<uint4*>(lds + lt * kPairTile + (ip + 8) * 8);
    l0[0] = make_uint4(w0[0], w0[1], w0[2], w0[3]);
    l0[1] = make_uint4(w0[4], w0[5], w0[6], w0[7]);
    l1[0] = make_uint4(w1[0], w1[1], w1[2], w1[3]);
    l1[1] = make_uint4(w1[4], w1[5], w1[6], w1[7]);
}

// ---- forward column pass (column role) ------------------------------------
// ya[u] = Y[u][p], yb[u] = Y[u][p+8] as int32.
template <typename S, int XF>
__device__ __forceinline__ void fwd_columns(const uint32_t* lds, int lt, int p, int32_t (&ya)[16],
                                            int32_t (&yb)[16]) {
    uint32_t w[16];
    const uint32_t* l = lds + lt * kPairTile + p;
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = l[k * 8];
    if constexpr (sizeof(S) == 1) {
        u16x2 z[16], y[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) z[k] = as_u16x2(w[k]);
        xf_fwd<XF>(z, y);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t t = as_u32(y[u]);
            ya[u] = sext_lo(t);
            yb[u] = sext_hi(t);
        }
        // the DC coefficient is the only one outside the signed 16-bit range
        if (p == 0) ya[0] = (int32_t)(as_u32(y[0]) & 0xffffu);
    } else {
        int32_t za[16], zb[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            za[k] = sext_lo(w[k]);
            zb[k] = sext_hi(w[k]);
        }
        xf_fwd<XF>(za, ya);
        xf_fwd<XF>(zb, yb);
    }
}

// ---- int32 block staging through LDS --------------------------------------
// Column role writes columns p and p+8 of a 16x16 int32 block.
__device__ __forceinline__ void lds_put_columns(uint32_t* lds, int lt, int p, const int32_t (&a)[16],
                                                const int32_t (&b)[16]) {
    int32_t* l = reinterpret_cast<int32_t*>(lds) + lt * kIntTile + p;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        l[u * kIntRow] = a[u];
        l[u * kIntRow + 8] = b[u];
    }
}

// Row role reads row i of the block.
__device__ __forceinline__ void lds_get_row(const uint32_t* lds, int lt, int i, int32_t (&r)[16]) {
    const int4* l = reinterpret_cast<const int4*>(lds + lt * kIntTile + i * kIntRow);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 w = l[k];
        r[4 * k] = w.x;
        r[4 * k + 1] = w.y;
        r[4 * k + 2] = w.z;
        r[4 * k + 3] = w.w;
    }
}

// Whole group: contiguous [ntile][16][16] int32 <-> LDS, 16-byte chunks,
// chunk c of the group = tile c/64, row (c/4)%16, column 4*(c%4).
template <int TPW>
__device__ __forceinline__ void lds_blocks_to_global(const uint32_t* lds, int tid, uint32_t ntile,
                                                     int32_t* out) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int c = tid + k * TPW * 8;
        const int t = c >> 6, u = (c >> 2) & 15, v4 = c & 3;
        if ((uint32_t)t < ntile)
            store16(reinterpret_cast<uint4*>(out) + c,
                    *reinterpret_cast<const uint4*>(lds + t * kIntTile + u * kIntRow + 4 * v4));
    }
}

// int16 blocks: chunk c (8 coefficients) = tile c/32, row (c/2)%16, half c%2.
template <int TPW>
__device__ __forceinline__ void lds_q_to_global(const uint32_t* lds, int tid, uint32_t ntile, int16_t* out) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = tid + k * TPW * 8;
        const int t = c >> 5, u = (c >> 1) & 15, h = c & 1;
        if ((uint32_t)t < ntile)
            store16(reinterpret_cast<uint4*>(out) + c,
                    *reinterpret_cast<const uint4*>(lds + t * kIntTile + u * kIntRow + 4 * h));
    }
}

// Column role writes int16 columns p, p+8 into the [tile][u][8 words] layout.
__device__ __forceinline__ void lds_put_q_columns(uint32_t* lds, int lt, int p, const int32_t (&qa)[16],
                                                  const int32_t (&qb)[16]) {
    int16_t* l = reinterpret_cast<int16_t*>(lds + lt * kIntTile) + p;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        l[u * 2 * kIntRow] = (int16_t)qa[u];
        l[u * 2 * kIntRow + 8] = (int16_t)qb[u];
    }
}

template <int TPW>
__device__ __forceinline__ void global_blocks_to_lds(const int32_t* in, int tid, uint32_t ntile, int rows,
                                                     int cols4, uint32_t* lds) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int c = tid + k * TPW * 8;
        const int t = c >> 6, u = (c >> 2) & 15, v4 = c & 3;
        int4 w = make_int4(0, 0, 0, 0);
        if ((uint32_t)t < ntile && u < rows && v4 < cols4) w = reinterpret_cast<const int4*>(in)[c];
        *reinterpret_cast<int4*>(lds + t * kIntTile + u * kIntRow + 4 * v4) = w;
    }
}

template <int TPW>
__device__ __forceinline__ void global_q_to_lds(const int16_t* in, int tid, uint32_t ntile, uint32_t* lds) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = tid + k * TPW * 8;
        const int t = c >> 5, u = (c >> 1) & 15, h = c & 1;
        uint4 w = make_uint4(0, 0, 0, 0);
        if ((uint32_t)t < ntile) w = reinterpret_cast<const uint4*>(in)[c];
        *reinterpret_cast<uint4*>(lds + t * kIntTile + u * kIntRow + 4 * h) = w;
    }
}

// Column role reads int32 columns p, p+8 (rows u < rows; others zero).
__device__ __forceinline__ void lds_get_columns(const uint32_t* lds, int lt, int p, int32_t (&a)[16],
                                                int32_t (&b)[16]) {
    const int32_t* l = reinterpret_cast<const int32_t*>(lds) + lt * kIntTile + p;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        a[u] = l[u * kIntRow];
        b[u] = l[u * kIntRow + 8];
    }
}

__device__ __forceinline__ void lds_get_q_columns(const uint32_t* lds, int lt, int p, int32_t (&a)[16],
                                                  int32_t (&b)[16]) {
    const int16_t* l = reinterpret_cast<const int16_t*>(lds + lt * kIntTile) + p;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        a[u] = l[u * 2 * kIntRow];
        b[u] = l[u * 2 * kIntRow + 8];
    }
}

// ---- coefficient domain ----------------------------------------------------
// Zonal retention with the S weights; r fixed at compile time (ZR >= 0) or
// at run time.
template <int ZR, int XF>
__device__ __forceinline__ void zonal_weights_cols(int p, int rr, int32_t (&a)[16], int32_t (&b)[16]) {
    const int r = ZR >= 0 ? ZR : rr;
    const int la = xf_lnorm<XF>(p), lb = xf_lnorm<XF>(p + 8);
    const bool ka = p < r, kb = p + 8 < r;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const bool ku = ZR >= 0 ? (u < ZR) : (u < r);
        const int su = 8 - xf_lnorm<XF>(u);
        a[u] = (ku && ka) ? (int32_t)((uint32_t)a[u] << (su - la)) : 0;
        b[u] = (ku && kb) ? (int32_t)((uint32_t)b[u] << (su - lb)) : 0;
    }
}

// Zig-zag retention of the first r coefficients with the S weights.
template <int XF>
__device__ __forceinline__ void zigzag_weights_cols(int p, int r, int32_t (&a)[16], int32_t (&b)[16]) {
    const int la = xf_lnorm<XF>(p), lb = xf_lnorm<XF>(p + 8);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int su = 8 - xf_lnorm<XF>(u);
        a[u] = zigzag_rank(u, p) < r ? (int32_t)((uint32_t)a[u] << (su - la)) : 0;
        b[u] = zigzag_rank(u, p + 8) < r ? (int32_t)((uint32_t)b[u] << (su - lb)) : 0;
    }
}

// The quantiser (or dequantiser) factors of columns p and p+8, per log2 d_u
// - 2.  Taken once, at the start of a group: their per-lane selects may be
// compiled into indexed loads of the table, and loading them early keeps
// that latency off the path from the forward transform to the quantiser.
struct ColFactors {
    float a[3], b[3];
};

__device__ __forceinline__ ColFactors col_factors(const Scale5& t, int p) {
    ColFactors f;
    column_factors(t, p, f.a);
    column_factors(t, p + 8, f.b);
    return f;
}

// Levels of columns p, p+8, saturated to int16 when SAT (without SAT the
// caller guarantees that they fit).
template <bool SAT>
__device__ __forceinline__ void quant_cols(const ColFactors& f, const int32_t (&a)[16], const int32_t (&b)[16],
                                           int32_t (&qa)[16], int32_t (&qb)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        qa[u] = round_away(__fmul_rn((float)a[u], f.a[log2_norm(u) - 2]));
        qb[u] = round_away(__fmul_rn((float)b[u], f.b[log2_norm(u) - 2]));
        if constexpr (SAT) {
            qa[u] = clamp_i32(qa[u], -32768, 32767);
            qb[u] = clamp_i32(qb[u], -32768, 32767);
        }
    }
}

__device__ __forceinline__ void dequant_cols(const ColFactors& f, int32_t (&a)[16], int32_t (&b)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        a[u] = round_away(__fmul_rn((float)a[u], f.a[log2_norm(u) - 2]));
        b[u] = round_away(__fmul_rn((float)b[u], f.b[log2_norm(u) - 2]));
    }
}

// ---- inverse ---------------------------------------------------------------
// Rounded, clamped sample kept in 8-fraction-bit fixed point: R (already
// holding the +128) clamped to [lo * 256, hi * 256 + 255].  The sample
// floor(R / 256) is then byte 1 of the result (uint8, in [0, 255]) or bytes
// 1-2 (int16, in [-255, 255] as a two's-complement halfword), so byte
// permutes pick it out with no shift.
template <typename S>
__device__ __forceinline__ int32_t out_fixed(int32_t R) {
    return clamp_i32(R, Samples<S>::kLo * 256, Samples<S>::kHi * 256 + 255);
}

// The samples of two out_fixed values as 16-bit lanes (a low, b high):
// uint8 zero-extended, int16 as is, the layout of pack_rows.
template <typename S>
__device__ __forceinline__ uint32_t pack_fixed_pair(int32_t a, int32_t b) {
    if constexpr (sizeof(S) == 1)
        return perm((uint32_t)b, (uint32_t)a, 0x0c050c01u);
    else
        return perm((uint32_t)b, (uint32_t)a, 0x06050201u);
}

// Stores the 16 samples of a row of out_fixed values.  `shared_lines`
// (uint8 planes): the plane's tile-group row segments begin or end inside
// 128-byte lines, which neighbouring groups then also write (see
// store16_rowpiece).
template <typename S>
__device__ __forceinline__ void store_row_fixed(char* p, const int32_t (&o)[16], bool shared_lines = false) {
    if constexpr (sizeof(S) == 1) {
        uint32_t ws[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t lo = perm((uint32_t)o[4 * k + 1], (uint32_t)o[4 * k], 0x0c0c0501u);
            const uint32_t hi = perm((uint32_t)o[4 * k + 3], (uint32_t)o[4 * k + 2], 0x05010c0cu);
            ws[k] = lo | hi;
        }
        store16_row(p, make_uint4(ws[0], ws[1], ws[2], ws[3]), shared_lines);
    } else {
        uint32_t ws[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) ws[k] = pack_fixed_pair<S>(o[2 * k], o[2 * k + 1]);
        store16(p, make_uint4(ws[0], ws[1], ws[2], ws[3]));
        store16(p + 16, make_uint4(ws[4], ws[5], ws[6], ws[7]));
    }
}

// int16 output rows leave through LDS: each thread stages its two packed
// rows (32 bytes each), then the workgroup stores 16-byte chunks with
// consecutive threads on consecutive chunks of one sample row across the
// group's tiles, so every store instruction writes whole contiguous lines.
// Stored straight from the row role, each row would go out as two pieces
// at a 32-byte stride, half of each line per instruction, which non-temporal
// stores do not merge.  Staged rows: [sample row][tile][8 words + 4 pad].
constexpr int kStageRowI16 = 12;

template <int TPW>
__device__ __forceinline__ void store_rows_i16(const GroupArgs& a, uint32_t g0, uint32_t ntile, uint32_t* lds,
                                               int lt, int ip, const int32_t (&r0)[16], const int32_t (&r1)[16]) {
    static_assert(16 * TPW * kStageRowI16 <= lds_words(TPW), "staging fits the group's LDS");
    uint4* s0 = reinterpret_cast<uint4*>(lds + (ip * TPW + lt) * kStageRowI16);
    uint4* s1 = reinterpret_cast<uint4*>(lds + ((ip + 8) * TPW + lt) * kStageRowI16);
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = pack_fixed_pair<int16_t>(r0[2 * k], r0[2 * k + 1]);
    s0[0] = make_uint4(w[0], w[1], w[2], w[3]);
    s0[1] = make_uint4(w[4], w[5], w[6], w[7]);
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = pack_fixed_pair<int16_t>(r1[2 * k], r1[2 * k + 1]);
    s1[0] = make_uint4(w[0], w[1], w[2], w[3]);
    s1[1] = make_uint4(w[4], w[5], w[6], w[7]);
    __syncthreads();
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = tid + i * TPW * 8;  // chunk: (sample row, tile, half)
        const int e = c >> 1, half = c & 1;
        const int row = e / TPW, t = e % TPW;
        if ((uint32_t)t < ntile) {
            const uint32_t g = g0 + (uint32_t)t;
            const uint32_t by = fdiv(g, a.bwdiv), bx = g - by * a.bw;
            char* p = const_cast<char*>(row_ptr<int16_t>(a.dst, by, bx, row)) + 16 * half;
            store16(p, *reinterpret_cast<const uint4*>(lds + e * kStageRowI16 + 4 * half));
        }
    }
}

// ---- per-image SSE accumulated across the groups of a workgroup ------------
constexpr uint32_t kNoImage = 0xffffffffu;

struct SseAcc {
    int32_t s;     // this thread's running sum for image `img`
    uint32_t img;  // image of the running sum (uniform over the workgroup)
};

__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Adds the workgroup's running sum to sse[img] with one atomic.  Called with
// uniform control flow.
template <int NTHREADS>
__device__ __forceinline__ void sse_flush(const SseAcc& acc, unsigned long long* sse, long long* red) {
    if (acc.img == kNoImage) return;
    const long long v = wave_sum64((long long)acc.s);
    const int tid = threadIdx.x;
    __syncthreads();  // a previous flush has finished reading `red`
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        long long t = 0;
#pragma unroll
        for (int w = 0; w < NTHREADS / 64; ++w) t += red[w];
        if (t) atomicAdd(sse + acc.img, (unsigned long long)t);
    }
}

// ---- the group ----------------------------------------------------------------
// Processes tiles g0 .. g0 + ntile - 1 (ntile <= TPW) of one plane.  Per-image
// SSE contributions go to sse[img(tile)] with img = tile_row / ipb.
// Row-role sample words of group (g0, ntile), for the forward input.
template <int TPW, typename S>
__device__ __forceinline__ void load_group_rows(const GroupArgs& a, uint32_t g0, uint32_t ntile, RowWords& w) {
    const int rlt = threadIdx.x % TPW, rip = threadIdx.x / TPW;
    const uint32_t rg = g0 + (uint32_t)rlt;
    const uint32_t rby = fdiv(rg, a.bwdiv), rbx = rg - rby * a.bw;
    load_rows<S>(a.src, rby, rbx, (uint32_t)rlt < ntile, rip, w.a0, w.a1, w.b0, w.b1);
}

// ---- zonal reconstruction with a compile-time zone ------------------------------
#ifndef ADCT_ZONE_MAX
#define ADCT_ZONE_MAX 16
#endif
// A uint8 zonal reconstruction from coefficients whose zone r x r is fixed at
// compile time reads, per tile, only the first ceil(r/4) 16-byte words of its
// first r coefficient rows, and the reference rows for the SSE.  For small r
// that is too little to keep the memory busy while the group's transforms
// run, so these words are requested a group ahead, into the `rows` of the
// group loop: reference rows in a0 / b0 (as load_rows leaves them for
// uint8), coefficient words in z.
template <typename S, typename M>
constexpr bool prefetch_zone() {
    return M::IN == kInY && M::MID == kMidZonal && M::ZR > 0 && M::ZR <= ADCT_ZONE_MAX && sizeof(S) == 1;
}

// Word i of a group's kept coefficient words: tile t, row u, word v4 of the
// row (kCols4 words per row, r rows per tile).
template <int ZR>
struct ZoneWords {
    static constexpr int kCols4 = (ZR + 3) / 4;
    static constexpr int kPerTile = ZR * kCols4;
    __device__ static void at(int i, int& t, int& u, int& v4) {
        t = i / kPerTile;
        const int rem = i - t * kPerTile;
        u = rem / kCols4;
        v4 = rem - u * kCols4;
    }
};

template <int TPW, typename S, typename M>
__device__ __forceinline__ void load_zone_words(const GroupArgs& a, uint32_t g0, uint32_t ntile, RowWords& w) {
    using Z = ZoneWords<M::ZR>;
    constexpr int kThreads = TPW * 8, kWords = TPW * Z::kPerTile;
    static_assert(kWords <= 8 * kThreads, "at most eight words per thread");
    const int tid = threadIdx.x;
    const uint4* in = reinterpret_cast<const uint4*>(static_cast<const int32_t*>(a.cin) + (int64_t)g0 * 256);
#pragma unroll
    for (int k = 0; k < (kWords + kThreads - 1) / kThreads; ++k) {
        const int i = tid + k * kThreads;
        int t, u, v4;
        Z::at(i, t, u, v4);
        w.z[k] = make_uint4(0, 0, 0, 0);
        if (i < kWords && (uint32_t)t < ntile) w.z[k] = in[t * 64 + u * 4 + v4];
    }
    if constexpr (M::SSE) {
        const int rlt = tid % TPW, rip = tid / TPW;
        const uint32_t rg = g0 + (uint32_t)rlt;
        const uint32_t rby = fdiv(rg, a.bwdiv), rbx = rg - rby * a.bw;
        uint4 unused0, unused1;  // uint8 rows fill a0 and b0 only
        load_rows<S>(a.ref, rby, rbx, (uint32_t)rlt < ntile, rip, w.a0, unused0, w.b0, unused1);
    }
}

// Writes the kept words into the group's LDS blocks.  The words outside the
// zone are left as they are: the zonal weights zero every coefficient
// outside r x r before it is used.
template <int TPW, typename M>
__device__ __forceinline__ void zone_words_to_lds(const RowWords& w, uint32_t* lds) {
    using Z = ZoneWords<M::ZR>;
    constexpr int kThreads = TPW * 8, kWords = TPW * Z::kPerTile;
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < (kWords + kThreads - 1) / kThreads; ++k) {
        const int i = tid + k * kThreads;
        int t, u, v4;
        Z::at(i, t, u, v4);
        if (i < kWords) *reinterpret_cast<uint4*>(lds + t * kIntTile + u * kIntRow + 4 * v4) = w.z[k];
    }
}

// `rows` holds this group's input rows (forward modes) or its zone words
// (prefetch_zone); once they are consumed, those of the next group (tiles
// g0n .. g0n + ntn - 1 of the plane of `an`, which may be another image's;
// ntn = 0 for none) are requested into it, so their latency overlaps this
// group's remaining work.
// `qs`, `dqs` must refer to kernel-argument or global memory: the per-class
// selects in column_factors may be compiled into indexed loads.
template <int TPW, typename S, typename M>
__device__ __forceinline__ void process_group(const GroupArgs& a, uint32_t g0, uint32_t ntile,
                                              uint32_t* lds, long long* red, SseAcc& acc, RowWords& rows,
                                              const GroupArgs& an, uint32_t g0n, uint32_t ntn, const Scale5& qs,
                                              const Scale5& dqs) {
    const int tid = threadIdx.x;
    const int rlt = tid % TPW, rip = tid / TPW;     // row role
    const int clt = tid >> 3, cp = tid & 7;         // column role
    const bool rok = (uint32_t)rlt < ntile;
    const uint32_t rg = g0 + (uint32_t)rlt;
    const uint32_t rby = fdiv(rg, a.bwdiv), rbx = rg - rby * a.bw;  // tile position (row role)

    uint32_t xk[16];   // packed input or reference samples (row role), for the SSE
    uint4 ra0, ra1, rb0, rb1;
    int32_t ya[16], yb[16];
    constexpr bool kQuant = M::MID == kMidQuant || M::MID == kMidQuantFit;
    constexpr bool kDequant = (kQuant && M::OUT != kOutNothing) || M::MID == kMidDequant;
    ColFactors qf{}, dqf{};
    if constexpr (kQuant) qf = col_factors(qs, cp);
    if constexpr (kDequant) dqf = col_factors(dqs, cp);

    // ---------------- input --------------------------------------------------
    if constexpr (M::IN == kInSamples) {
        fwd_rows<S, M::XF>(rows, rlt, rip, lds, xk);
        if (ntn) load_group_rows<TPW, S>(an, g0n, ntn, rows);
        __syncthreads();
        fwd_columns<S, M::XF>(lds, clt, cp, ya, yb);
    } else if constexpr (prefetch_zone<S, M>()) {
        zone_words_to_lds<TPW, M>(rows, lds);
        if constexpr (M::SSE) {
            ra0 = rows.a0;
            rb0 = rows.b0;
            ra1 = rb1 = make_uint4(0, 0, 0, 0);
        }
        __syncthreads();
        if (ntn) load_zone_words<TPW, S, M>(an, g0n, ntn, rows);
        lds_get_columns(lds, clt, cp, ya, yb);
    } else {
        if constexpr (M::SSE) {
            // prefetch the reference rows so their latency overlaps the rest
            load_rows<S>(a.ref, rby, rbx, rok, rip, ra0, ra1, rb0, rb1);
        }
        if constexpr (M::IN == kInQ) {
            global_q_to_lds<TPW>(static_cast<const int16_t*>(a.cin) + (int64_t)g0 * 256, tid, ntile, lds);
            __syncthreads();
            lds_get_q_columns(lds, clt, cp, ya, yb);
        } else {
            int rows = 16, cols4 = 4;
            if constexpr (M::MID == kMidZonal) {
                const int r = M::ZR >= 0 ? M::ZR : a.r;
                rows = r;
                cols4 = (r + 3) >> 2;
            } else if constexpr (M::MID == kMidZigzag) {
                rows = zigzag_extent(a.r);
                cols4 = (rows + 3) >> 2;
            }
            global_blocks_to_lds<TPW>(static_cast<const int32_t*>(a.cin) + (int64_t)g0 * 256, tid, ntile,
                                      rows, cols4, lds);
            __syncthreads();
            lds_get_columns(lds, clt, cp, ya, yb);
        }
    }

    // ---------------- coefficient domain ----------------------------------------
    // (a.cout and a.sse are uniform: a null pointer skips that output)
    if constexpr (M::STORE == kStoreY) {
        if (a.cout) {
            __syncthreads();
            lds_put_columns(lds, clt, cp, ya, yb);
            __syncthreads();
            lds_blocks_to_global<TPW>(lds, tid, ntile, static_cast<int32_t*>(a.cout) + (int64_t)g0 * 256);
        }
    }
    if constexpr (M::MID == kMidQuant || M::MID == kMidQuantFit) {
        // uint8 samples give |Y s_u s_v| <= 16 * 255 = 4080 and 1 / Delta <
        // 1.6, so their levels always fit int16
        constexpr bool sat = M::MID == kMidQuant && sizeof(S) == 2;
        int32_t qa[16], qb[16];
        quant_cols<sat>(qf, ya, yb, qa, qb);
        if constexpr (M::STORE == kStoreQ) {
            if (a.cout) {
                __syncthreads();
                lds_put_q_columns(lds, clt, cp, qa, qb);
                __syncthreads();
                lds_q_to_global<TPW>(lds, tid, ntile, static_cast<int16_t*>(a.cout) + (int64_t)g0 * 256);
            }
        }
        if constexpr (M::OUT != kOutNothing) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                ya[u] = qa[u];
                yb[u] = qb[u];
            }
            dequant_cols(dqf, ya, yb);
        }
    } else if constexpr (M::MID == kMidDequant) {
        dequant_cols(dqf, ya, yb);
    } else if constexpr (M::MID == kMidZonal) {
        zonal_weights_cols<M::ZR, M::XF>(cp, a.r, ya, yb);
    } else if constexpr (M::MID == kMidZigzag) {
        zigzag_weights_cols<M::XF>(cp, a.r, ya, yb);
    }

    if constexpr (M::OUT == kOutNothing) return;

    // ---------------- inverse ------------------------------------------------------
    if constexpr (M::OUT == kOutSamples) {
        if (cp == 0) ya[0] += 128;  // rounding offset, reaches every sample
    }
    {
        int32_t qa[16], qb[16];
        xf_inv<M::XF>(ya, qa);
        xf_inv<M::XF>(yb, qb);
        __syncthreads();
        lds_put_columns(lds, clt, cp, qa, qb);
        __syncthreads();
    }
    int32_t r0[16], r1[16];
    {
        int32_t q[16];
        lds_get_row(lds, rlt, rip, q);
        xf_inv<M::XF>(q, r0);
        lds_get_row(lds, rlt, rip + 8, q);
        xf_inv<M::XF>(q, r1);
    }
    if constexpr (M::OUT == kOutBlocks) {
        // the blocks leave through LDS as whole contiguous chunks (stored
        // from the row role, a lane's 64-byte row would go out as four
        // pieces, one per instruction, each a quarter of a line)
        __syncthreads();  // every read of the inverse transpose is done
        int4* l0 = reinterpret_cast<int4*>(lds + rlt * kIntTile + rip * kIntRow);
        int4* l1 = reinterpret_cast<int4*>(lds + rlt * kIntTile + (rip + 8) * kIntRow);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            l0[k] = make_int4(r0[4 * k], r0[4 * k + 1], r0[4 * k + 2], r0[4 * k + 3]);
            l1[k] = make_int4(r1[4 * k], r1[4 * k + 1], r1[4 * k + 2], r1[4 * k + 3]);
        }
        __syncthreads();
        lds_blocks_to_global<TPW>(lds, tid, ntile, a.bout + (int64_t)g0 * 256);
        return;
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            r0[j] = out_fixed<S>(r0[j]);
            r1[j] = out_fixed<S>(r1[j]);
        }
        if constexpr (sizeof(S) == 1) {
            // one 16-byte piece per row: the lanes of a sample row store one
            // contiguous run
            // groups of whole lines (base, pitch and row length multiples of
            // 128 bytes) keep the streaming stores, which leave the cache to
            // inputs that a later call may read again
            const bool shared_lines = shares_lines(a.dst.data, a.dst.pitch, (uint64_t)a.bw * 16u);
            if (rok) {
                char* pa = const_cast<char*>(row_ptr<S>(a.dst, rby, rbx, rip));
                store_row_fixed<S>(pa, r0, shared_lines);
                store_row_fixed<S>(pa + 8 * a.dst.pitch, r1, shared_lines);
            }
        } else {
            __syncthreads();  // every read of the inverse transpose is done
            store_rows_i16<TPW>(a, g0, ntile, lds, rlt, rip, r0, r1);
        }
        if constexpr (M::SSE) {
          if (a.sse) {
            if constexpr (M::IN != kInSamples) pack_rows<S>(ra0, ra1, rb0, rb1, xk);
            int32_t s = rok ? pair_sse<S>(r0, r1, xk) : 0;
            // a group inside one image adds to the workgroup's running sum
            // (flushed when the image changes); a group that straddles
            // images adds per thread
            const uint32_t img0 = fdiv(fdiv(g0, a.bwdiv), a.ipbdiv);
            const uint32_t img1 = fdiv(fdiv(g0 + ntile - 1u, a.bwdiv), a.ipbdiv);
            if (img0 != acc.img) {
                sse_flush<TPW * 8>(acc, a.sse, red);
                acc.s = 0;
                acc.img = img0;
            }
            if (img0 == img1) {
                acc.s += s;
            } else if (img1 == img0 + 1u) {
                // the group ends in the next image: close img0 with this
                // group's part of it, then start img1 with the rest
                const bool first = !rok || fdiv(rby, a.ipbdiv) == img0;
                acc.s += first ? s : 0;
                sse_flush<TPW * 8>(acc, a.sse, red);
                acc.s = first ? 0 : s;
                acc.img = img1;
            } else if (rok && s != 0) {
                // images smaller than a group: one atomic per thread
                atomicAdd(a.sse + fdiv(rby, a.ipbdiv), (unsigned long long)s);
            }
          }
        }
    }
}

}  // namespace adct

namespace adct {

#ifndef ADCT_TPW
#define ADCT_TPW 16
#endif
// Tiles per workgroup of the one-group-per-workgroup kernels.
constexpr int kTPW = ADCT_TPW;
static_assert(kTPW >= 8 && (kTPW & (kTPW - 1)) == 0, "TPW must be a power of two >= 8");

#ifndef ADCT_SSE_SPREAD
#define ADCT_SSE_SPREAD 4
#endif
// Workgroups of a launch that accumulates per-image SSE over large images
// (more than kSseSpreadMin chunks per image) are dealt over the plane in
// kSseSpread interleaved streams, so that the workgroups resident at one
// time add to the SSE of several images instead of queueing on the atomics
// of one or two.  Few streams suffice for that, and each stream stays a
// sequential sweep of its part of the plane: with 256 streams the
// resident workgroups touched 256 places at once and a 25.8 GB launch
// streamed 4.2 TB/s; 16, 8, 4 and 2 streams gave 5.55, 5.77, 5.84 and
// 5.74 TB/s (no interleave 5.65), and 2 streams let the video frames'
// atomics queue again.
#ifndef ADCT_SSE_SPREAD_MIN
#define ADCT_SSE_SPREAD_MIN 64
#endif
constexpr uint32_t kSseSpread = ADCT_SSE_SPREAD;
constexpr uint32_t kSseSpreadMin = ADCT_SSE_SPREAD_MIN;
static_assert((kSseSpread & (kSseSpread - 1)) == 0, "the stream count is a power of two");
// A launch that writes uint8 rows whose tile-group segments share 128-byte
// lines with their neighbours' (see shares_lines) deals its chunks over
// kXcdRegions contiguous regions instead: workgroups go to the 8 XCDs in
// turn, so each XCD sweeps one region and the two parts of a shared line
// meet in its L2, where the cached row stores merge them.  On 4096 images
// of 1008^2 that took the encoder from 5.23 to 5.61 TB/s; on planes of whole
// lines it was 1-2 % slower than the order above, which they keep.
constexpr uint32_t kXcdRegions = 8;

// `gpw` consecutive groups (a chunk) per workgroup; the per-image SSE is
// reduced in registers across them.  spread_rows = 0: workgroup b takes
// chunk b; otherwise the grid is n x spread_rows, n = 2^spread_log2 streams
// (kSseSpread or kXcdRegions), and workgroup b takes chunk (b % n) *
// spread_rows + b / n (workgroups past the last chunk exit at once).
// PF = false is the form for gpw == 1: with no next group to prefetch, no
// registers are held for one while the group is coded, which keeps the SSE
// modes at 5 waves per SIMD instead of 4.
// `qs`, `dqs`: as for process_group.
template <int TPW, typename S, typename M, bool PF>
__device__ __forceinline__ void group_chunk(const GroupArgs& a, uint32_t nblk, uint32_t gpw, uint32_t spread_rows,
                                            uint32_t spread_log2,
                                            uint32_t b, uint32_t* lds, long long* red, const Scale5& qs,
                                            const Scale5& dqs) {
    SseAcc acc{0, kNoImage};
    RowWords rows;
    const uint32_t chunk = spread_rows ? (b & ((1u << spread_log2) - 1u)) * spread_rows + (b >> spread_log2) : b;
    uint32_t g0 = chunk * gpw * (uint32_t)TPW;
    if (g0 >= nblk) return;
    if constexpr (M::IN == kInSamples) load_group_rows<TPW, S>(a, g0, min((uint32_t)TPW, nblk - g0), rows);
    if constexpr (prefetch_zone<S, M>()) load_zone_words<TPW, S, M>(a, g0, min((uint32_t)TPW, nblk - g0), rows);
    if constexpr (PF) {
        const uint32_t gend = min(nblk, g0 + gpw * (uint32_t)TPW);
        for (uint32_t k = 0; g0 < gend; ++k, g0 += (uint32_t)TPW) {
            if (k) __syncthreads();  // the previous group's LDS reads are done
            const uint32_t g0n = g0 + (uint32_t)TPW;
            const uint32_t ntn = g0n < gend ? min((uint32_t)TPW, gend - g0n) : 0u;
            process_group<TPW, S, M>(a, g0, min((uint32_t)TPW, nblk - g0), lds, red, acc, rows, a, g0n, ntn, qs,
                                     dqs);
        }
    } else {
        process_group<TPW, S, M>(a, g0, min((uint32_t)TPW, nblk - g0), lds, red, acc, rows, a, 0u, 0u, qs, dqs);
    }
    if constexpr (M::SSE) {
        if (a.sse) sse_flush<TPW * 8>(acc, a.sse, red);
    }
}

template <int TPW, typename S, typename M, bool PF>
__global__ __launch_bounds__(TPW * 8) void k_group(GroupArgs a, uint32_t nblk, uint32_t gpw, uint32_t spread_rows,
                                                   uint32_t spread_log2) {
    __shared__ uint32_t lds[lds_words(TPW)];
    __shared__ long long red[TPW * 8 / 64];
    group_chunk<TPW, S, M, PF>(a, nblk, gpw, spread_rows, spread_log2, blockIdx.x, lds, red, a.qs, a.dqs);
}

// Several planes of one mode in one launch: plane i takes the workgroups
// from first_wg (ascending) up to the next plane's, and runs them as
// k_group would run its own launch over that plane alone.  Every plane of
// the launch has the same quantiser (taken from plane 0).
constexpr int kMaxPlanes = 8;
struct PlaneLaunch {
    GroupArgs a;
    uint32_t nblk, gpw, spread_rows, spread_log2, first_wg;
};
struct PlaneSet {
    PlaneLaunch p[kMaxPlanes];
    uint32_t n;
};

template <int TPW, typename S, typename M, bool PF>
__global__ __launch_bounds__(TPW * 8) void k_group_planes(PlaneSet ps) {
    __shared__ uint32_t lds[lds_words(TPW)];
    __shared__ long long red[TPW * 8 / 64];
    uint32_t i = 0;
#pragma unroll
    for (uint32_t k = 1; k < (uint32_t)kMaxPlanes; ++k)
        if (k < ps.n && blockIdx.x >= ps.p[k].first_wg) i = k;
    const PlaneLaunch& pl = ps.p[i];
    group_chunk<TPW, S, M, PF>(pl.a, pl.nblk, pl.gpw, pl.spread_rows, pl.spread_log2, blockIdx.x - pl.first_wg, lds,
                               red, ps.p[0].a.qs,
                               ps.p[0].a.dqs);
}

#ifndef ADCT_TARGET_WGS
#define ADCT_TARGET_WGS 1048576
#endif
#ifndef ADCT_MAX_GPW
#define ADCT_MAX_GPW 32
#endif
// Groups per workgroup for a plain launch over nblk tiles: one group per
// workgroup up to a million workgroups (16.7 M tiles), then as few more as
// that allows.  Short chunks keep the workgroups resident at one time on a
// narrow band of the planes: measured on MI355X on 2048 to 16384 images of
// 512 x 512, four or more groups per workgroup stream 7-11 % slower than one
// or two (16384 images: 5.19 TB/s with 8 groups per workgroup, 5.84 with 1).
inline uint32_t groups_per_wg(uint32_t nblk) {
    const uint32_t groups = (nblk + kTPW - 1) / kTPW;
    uint32_t g = (groups + ADCT_TARGET_WGS - 1) / ADCT_TARGET_WGS;
    return g < 1 ? 1 : (g > ADCT_MAX_GPW ? ADCT_MAX_GPW : g);
}

#ifndef ADCT_ZONE_GPW
#define ADCT_ZONE_GPW 2
#endif
#ifndef ADCT_SSE_GPW
#define ADCT_SSE_GPW 2
#endif
// Groups per workgroup, at least, of the plain launches that add to the SSE
// of images of at most kSseSpreadMin groups.  A workgroup adds its sum to its
// image's slot with one device-scope atomic when it ends.  The workgroups of
// such an image run side by side and end together: with one group per
// workgroup the 64 atomics of each 512 x 512 image cost the headline encoder
// 7 % (288 against 267 us per call with the atomic left out, 1024 such
// images), and two groups per workgroup, half the atomics, took it to 270-274
// us (quantising and zig-zag encoders 7 % faster too).  Larger images are
// dealt in interleaved streams, which spread their atomics out in time; two
// groups per workgroup made them slower (4096 images of 1024^2 4.40 against
// 4.60 ms, 1008^2 4.45 against 4.90 ms, the video frames 223 against 237 us).
constexpr uint32_t kSseGpw = ADCT_SSE_GPW;
inline bool sse_gathers(bool sse, uint32_t image_tiles) {
    return sse && image_tiles / (uint32_t)kTPW <= kSseSpreadMin;
}
static_assert(kSseGpw >= 1 && kSseGpw <= ADCT_MAX_GPW, "groups per workgroup");

// Groups per workgroup, at least, of the launches that request their zone
// words a group ahead (prefetch_zone): with one group there is nothing to
// request ahead.
constexpr uint32_t kZoneGpw = ADCT_ZONE_GPW;
static_assert(kZoneGpw >= 1 && kZoneGpw <= ADCT_MAX_GPW, "groups per workgroup");

}  // namespace adct
