// 16-point multiplierless approximate DCT: the 1D butterflies.
//
// T (Section 2.1) is applied through its sparse factorisation
// T = P2 M4 M3 M2 P1 M1 (Section 2.2).  The stages are folded by hand into
// one straight-line dataflow: M1 is the outer butterfly (16 add/sub), M2 the
// two 8-point butterflies (16), M3 the two 4-point butterflies (8; its -I4
// blocks are absorbed into operand order), M4 the final 2-point butterflies
// (4; its sign-only rows absorbed likewise), and P1/P2 are only the naming
// of outputs.  The result is exactly 44 additions/subtractions, no
// negations, multiplies or shifts.  Outputs become final at different depths:
// eight after two stages, four after three, four after four.
//
// The inverse direction applies T^T = M1 P1^T M2 M3 M4 P2^T (all M_i are
// symmetric): the same graph mirrored, again 44 additions/subtractions.
//
// V may be any type with exact + and - over the values it carries
// (int32, or a packed pair of int16 lanes, or float on integers < 2^24).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adct {

// log2 of d_k = (T T^T)_kk = (16,16,4,8,8,16,4,4,16,4,4,8,8,4,4,4), packed
// two bits per k as (log2 d_k - 2).
constexpr uint32_t kLog2NormPacked =
    (2u << 0) | (2u << 2) | (0u << 4) | (1u << 6) | (1u << 8) | (2u << 10) | (0u << 12) |
    (0u << 14) | (2u << 16) | (0u << 18) | (0u << 20) | (1u << 22) | (1u << 24) | (0u << 26) |
    (0u << 28) | (0u << 30);

__host__ __device__ constexpr int log2_norm(int k) {
    return (int)((kLog2NormPacked >> (2 * k)) & 3u) + 2;
}

// Rank of coefficient (u, v) (u vertical, v horizontal frequency) in the
// zig-zag scan of a 16x16 block, the retention order of Section 3.1: the
// JPEG scan extended to 16x16, anti-diagonal s = u + v after anti-diagonal,
// u rising on odd s and falling on even s.
__host__ __device__ constexpr int zigzag_rank(int u, int v) {
    const int s = u + v;
    const int base = s < 16 ? s * (s + 1) / 2 : 256 - (31 - s) * (32 - s) / 2;
    const int lo = s < 16 ? 0 : s - 15, hi = s < 16 ? s : 15;
    return base + ((s & 1) ? u - lo : hi - u);
}

// Rows (and columns) of a block that hold the first r zig-zag coefficients.
__host__ __device__ constexpr int zigzag_extent(int r) {
    if (r <= 0) return 0;
    int s = 0;
    while (s < 15 && (s + 1) * (s + 2) / 2 < r) ++s;  // first r ranks lie on diagonals 0..s
    return s + 1;
}

// X = T x.
template <typename V>
__host__ __device__ __forceinline__ void fwd16(const V (&x)[16], V (&X)[16]) {
    // M1: outer butterfly
    const V a0 = x[0] + x[15], a1 = x[1] + x[14], a2 = x[2] + x[13], a3 = x[3] + x[12];
    const V a4 = x[4] + x[11], a5 = x[5] + x[10], a6 = x[6] + x[9], a7 = x[7] + x[8];
    const V a8 = x[7] - x[8], a9 = x[6] - x[9], a10 = x[5] - x[10], a11 = x[4] - x[11];
    const V a12 = x[3] - x[12], a13 = x[2] - x[13], a14 = x[1] - x[14], a15 = x[0] - x[15];
    // M2 (after P1): the even half and the odd half, 8-point butterflies;
    // the difference outputs are final coefficients.
    const V b0 = a0 + a7, b1 = a1 + a6, b2 = a2 + a5, b3 = a3 + a4;
    X[2] = a0 - a7;
    X[10] = a6 - a1;
    X[6] = a5 - a2;
    X[14] = a4 - a3;
    const V b8 = a8 + a9, b9 = a11 + a10, b10 = a12 + a13, b11 = a15 + a14;
    X[7] = a8 - a9;
    X[15] = a10 - a11;
    X[9] = a12 - a13;
    X[13] = a15 - a14;
    // M3: 4-point butterflies
    const V c0 = b0 + b3, c1 = b1 + b2, c8 = b8 + b11, c9 = b9 + b10;
    X[4] = b0 - b3;
    X[12] = b2 - b1;
    X[3] = b11 - b8;
    X[11] = b10 - b9;
    // M4: 2-point butterflies
    X[0] = c0 + c1;
    X[8] = c0 - c1;
    X[1] = c8 + c9;
    X[5] = c8 - c9;
}

// x = T^T X.
template <typename V>
__host__ __device__ __forceinline__ void inv16(const V (&X)[16], V (&x)[16]) {
    // M4 (after P2^T)
    const V c0 = X[0] + X[8], c1 = X[0] - X[8], c8 = X[1] + X[5], c9 = X[1] - X[5];
    // M3
    const V b0 = c0 + X[4], b3 = c0 - X[4], b1 = c1 - X[12], b2 = c1 + X[12];
    const V b8 = c8 - X[3], b11 = c8 + X[3], b9 = c9 - X[11], b10 = c9 + X[11];
    // M2
    const V p0 = b0 + X[2], p7 = b0 - X[2], p1 = b1 - X[10], p6 = b1 + X[10];
    const V p2 = b2 - X[6], p5 = b2 + X[6], p3 = b3 - X[14], p4 = b3 + X[14];
    const V p8 = b8 + X[7], p15 = b8 - X[7], p9 = b9 - X[15], p14 = b9 + X[15];
    const V p10 = b10 + X[9], p13 = b10 - X[9], p11 = b11 + X[13], p12 = b11 - X[13];
    // P1^T, then M1
    x[0] = p0 + p11;
    x[15] = p0 - p11;
    x[1] = p1 + p12;
    x[14] = p1 - p12;
    x[2] = p2 + p13;
    x[13] = p2 - p13;
    x[3] = p3 + p10;
    x[12] = p3 - p10;
    x[4] = p4 + p9;
    x[11] = p4 - p9;
    x[5] = p5 + p14;
    x[10] = p5 - p14;
    x[6] = p6 + p15;
    x[9] = p6 - p15;
    x[7] = p7 + p8;
    x[8] = p7 - p8;
}

// The natural-order Walsh-Hadamard transform of order 16 (H[k][j] =
// (-1)^popcount(k & j)), the WHT row of Table 2, used as a comparison
// transform: butterflies (a + b, a - b) at strides 8, 4, 2, 1, 64 additions.
// H^T = H, so the same dataflow is its inverse (up to the factor 16).
template <typename V>
__host__ __device__ __forceinline__ void wht16(const V (&x)[16], V (&X)[16]) {
    V a[16], b[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = x[i] + x[i + 8];
        a[i + 8] = x[i] - x[i + 8];
    }
#pragma unroll
    for (int i = 0; i < 16; i += 8)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b[i + j] = a[i + j] + a[i + j + 4];
            b[i + j + 4] = a[i + j] - a[i + j + 4];
        }
#pragma unroll
    for (int i = 0; i < 16; i += 4)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            a[i + j] = b[i + j] + b[i + j + 2];
            a[i + j + 2] = b[i + j] - b[i + j + 2];
        }
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
        X[i] = a[i] + a[i + 1];
        X[i + 1] = a[i] - a[i + 1];
    }
}

// Transform selection of the group kernel: the proposed T (default) or the
// WHT.  lnorm is log2 of the squared row norm d_k (T: from the table above;
// WHT: 16 for every row).
enum Xform { kXfProposed = 0, kXfWht = 1 };

template <int XF, typename V>
__host__ __device__ __forceinline__ void xf_fwd(const V (&x)[16], V (&X)[16]) {
    if constexpr (XF == kXfWht)
        wht16(x, X);
    else
        fwd16(x, X);
}

template <int XF, typename V>
__host__ __device__ __forceinline__ void xf_inv(const V (&X)[16], V (&x)[16]) {
    if constexpr (XF == kXfWht)
        wht16(X, x);
    else
        inv16(X, x);
}

template <int XF>
__host__ __device__ constexpr int xf_lnorm(int k) {
    return XF == kXfWht ? 4 : log2_norm(k);
}

}  // namespace adct
