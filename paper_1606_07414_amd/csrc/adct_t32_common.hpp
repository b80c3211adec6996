// The 32-point extension of the approximation (Section 5 extends the
// 16-point approach to 32 points by the construction that builds T from two
// 8-point blocks): T32 = P32 diag(T, T) B32.  B32 folds the input into the
// sums x_j + x_{31-j} and the differences x_j - x_{31-j} (32 additions), T
// (the 44-addition dataflow of Section 2.2) transforms each half, and P32
// interleaves the results: coefficient 2k from the sums, 2k + 1 from the
// differences.  120 additions, no negations.
//
// With d16 the diagonal of T T^T, T32 T32^T = diag(2 d16[u / 2]), entries 8,
// 16 or 32; the codec's fixed point carries 10 fractional bits (weights
// 1024 / (d_u d_v) in {1, ..., 16}).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "adct_butterfly.hpp"

namespace adct {

// log2 of row u's squared norm: 3, 4 or 5.
__host__ __device__ constexpr int l32(int u) { return 1 + log2_norm(u >> 1); }

// X = T32 x.
template <typename V>
__host__ __device__ __forceinline__ void fwd32(const V (&x)[32], V (&X)[32]) {
    V s[16], d[16], ys[16], yd[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        s[j] = x[j] + x[31 - j];
        d[j] = x[j] - x[31 - j];
    }
    fwd16(s, ys);
    fwd16(d, yd);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        X[2 * k] = ys[k];
        X[2 * k + 1] = yd[k];
    }
}

// x = T32^T X: T^T on the even and on the odd coefficients, then B32^T
// (x_j = s_j + d_j, x_{31-j} = s_j - d_j).
template <typename V>
__host__ __device__ __forceinline__ void inv32(const V (&X)[32], V (&x)[32]) {
    V ys[16], yd[16], s[16], d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        ys[k] = X[2 * k];
        yd[k] = X[2 * k + 1];
    }
    inv16(ys, s);
    inv16(yd, d);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        x[j] = s[j] + d[j];
        x[31 - j] = s[j] - d[j];
    }
}

// Quantiser and dequantiser factors of the 32x32 codec per class
// c = log2 d_u + log2 d_v - 6 (d_u d_v = 2^(c+6)): qs = fp32(s_u s_v / Delta),
// dqs = fp32(1024 Delta s_u s_v), Delta = 2^((QP - 4) / 6).  False if QP is
// out of range.
inline bool quant_scales32(int qp, float* qs, float* dqs) {
    if (qp < 0 || qp > 63) return false;
    const double delta = std::exp2((qp - 4) / 6.0);
    for (int c = 0; c < 5; ++c) {
        const double ss = 1.0 / std::sqrt((double)(1 << (c + 6)));
        if (qs) qs[c] = (float)(ss / delta);
        if (dqs) dqs[c] = (float)(1024.0 * delta * ss);
    }
    return true;
}

}  // namespace adct
