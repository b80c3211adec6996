// The 64-point extension of the approximation: the construction that builds
// T from two 8-point blocks (Section 2.1), taken two levels up through the
// 32-point extension: T64 = P64 diag(T32, T32) B64.  B64 folds the input
// into the sums x_j + x_{63-j} and the differences x_j - x_{63-j} (64
// additions), T32 (120 additions) transforms each half, and P64 interleaves
// the results: coefficient 2k from the sums, 2k + 1 from the differences.
// 304 additions, no negations.
//
// T64 T64^T = diag(2 d32[u / 2]), entries 16, 32 or 64; the codec's fixed
// point carries 12 fractional bits (weights 4096 / (d_u d_v) in {1, ..., 16}).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include "adct_t32_common.hpp"

namespace adct {

// log2 of row u's squared norm: 4, 5 or 6.
__host__ __device__ constexpr int l64(int u) { return 1 + l32(u >> 1); }

// X = T64 x.
template <typename V>
__host__ __device__ __forceinline__ void fwd64(const V (&x)[64], V (&X)[64]) {
    V s[32], d[32], ys[32], yd[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        s[j] = x[j] + x[63 - j];
        d[j] = x[j] - x[63 - j];
    }
    fwd32(s, ys);
    fwd32(d, yd);
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        X[2 * k] = ys[k];
        X[2 * k + 1] = yd[k];
    }
}

// x = T64^T X: T32^T on the even and on the odd coefficients, then B64^T
// (x_j = s_j + d_j, x_{63-j} = s_j - d_j).
template <typename V>
__host__ __device__ __forceinline__ void inv64(const V (&X)[64], V (&x)[64]) {
    V ys[32], yd[32], s[32], d[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        ys[k] = X[2 * k];
        yd[k] = X[2 * k + 1];
    }
    inv32(ys, s);
    inv32(yd, d);
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        x[j] = s[j] + d[j];
        x[63 - j] = s[j] - d[j];
    }
}

// Quantiser and dequantiser factors of the 64x64 codec per class
// c = log2 d_u + log2 d_v - 8 (d_u d_v = 2^(c+8)): qs = fp32(s_u s_v / Delta),
// dqs = fp32(4096 Delta s_u s_v), Delta = 2^((QP - 4) / 6).  False if QP is
// out of range.
inline bool quant_scales64(int qp, float* qs, float* dqs) {
    if (qp < 0 || qp > 63) return false;
    const double delta = std::exp2((qp - 4) / 6.0);
    for (int c = 0; c < 5; ++c) {
        const double ss = 1.0 / std::sqrt((double)(1 << (c + 8)));
        if (qs) qs[c] = (float)(ss / delta);
        if (dqs) dqs[c] = (float)(4096.0 * delta * ss);
    }
    return true;
}

}  // namespace adct
