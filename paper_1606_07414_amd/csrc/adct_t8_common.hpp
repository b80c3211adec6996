// The 8-point approximation T8 (Section 2.1): its butterflies and quantiser
// factors, shared by the 8x8 codec and the mixed 8/16-point codec.
//
// T8 is the sum-path block of the factorisation of Section 2.2: the even
// rows of T act on the folded input x_j + x_{15-j} only, and their left
// halves are T8 (T8[k][j] = T[2k][j]).  Its dataflow is the even path of the
// 16-point one: 8 + 4 + 2 = 14 additions, no negations.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace adct {

// log2 d_k of T8's rows: d = diag(T8 T8^T) = (8, 2, 4, 2, 8, 2, 4, 2)
__host__ __device__ constexpr int l8(int k) { return (k & 3) == 0 ? 3 : (k & 3) == 2 ? 2 : 1; }

// X = T8 x (14 add/sub).
template <typename V>
__host__ __device__ __forceinline__ void fwd8(const V (&x)[8], V (&y)[8]) {
    const V b0 = x[0] + x[7], b1 = x[1] + x[6], b2 = x[2] + x[5], b3 = x[3] + x[4];
    y[1] = x[0] - x[7];
    y[3] = x[5] - x[2];
    y[5] = x[6] - x[1];
    y[7] = x[4] - x[3];
    const V c0 = b0 + b3, c1 = b1 + b2;
    y[2] = b0 - b3;
    y[6] = b2 - b1;
    y[0] = c0 + c1;
    y[4] = c0 - c1;
}

// x = T8^T y (the transposed dataflow, 14 add/sub).
template <typename V>
__host__ __device__ __forceinline__ void inv8(const V (&y)[8], V (&x)[8]) {
    const V c0 = y[0] + y[4], c1 = y[0] - y[4];
    const V b0 = c0 + y[2], b3 = c0 - y[2], b1 = c1 - y[6], b2 = c1 + y[6];
    x[0] = b0 + y[1];
    x[7] = b0 - y[1];
    x[1] = b1 - y[5];
    x[6] = b1 + y[5];
    x[2] = b2 - y[3];
    x[5] = b2 + y[3];
    x[3] = b3 - y[7];
    x[4] = b3 + y[7];
}

// Quantiser and dequantiser factors of the 8x8 codec per class
// c = log2 d_u + log2 d_v - 2 (d_u d_v = 2^(c+2)):  qs = fp32(s_u s_v / Delta),
// dqs = fp32(64 Delta s_u s_v), Delta = 2^((QP - 4) / 6).  False if QP is out
// of range.
inline bool quant_scales8(int qp, float* qs, float* dqs) {
    if (qp < 0 || qp > 63) return false;
    const double delta = std::exp2((qp - 4) / 6.0);
    for (int c = 0; c < 5; ++c) {
        const double ss = 1.0 / std::sqrt((double)(1 << (c + 2)));
        if (qs) qs[c] = (float)(ss / delta);
        if (dqs) dqs[c] = (float)(64.0 * delta * ss);
    }
    return true;
}

}  // namespace adct
