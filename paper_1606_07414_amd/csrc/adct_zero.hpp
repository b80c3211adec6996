// Clearing of several per-image SSE arrays in one launch, for the calls
// that code several planes at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adct {

// Up to N arrays: row y of the grid clears array y (rows of n[y] == 0 or at
// or past `count` do nothing).
template <int N>
struct ZeroSet {
    unsigned long long* p[N];
    uint32_t n[N];
    uint32_t count;
};

template <int N>
__global__ __launch_bounds__(256) void k_zero_sets(ZeroSet<N> z) {
    const uint32_t y = blockIdx.y, t = blockIdx.x * 256u + threadIdx.x;
    if (y < z.count && t < z.n[y]) z.p[y][t] = 0ull;
}

// Launches the clear of z's arrays on s (nothing when none is set).
template <int N>
inline void clear_sets(const ZeroSet<N>& z, hipStream_t s) {
    uint32_t most = 0;
    for (uint32_t i = 0; i < z.count; ++i) most = z.n[i] > most ? z.n[i] : most;
    if (most) hipLaunchKernelGGL(k_zero_sets<N>, dim3((most + 255) / 256, z.count), dim3(256), 0, s, z);
}

}  // namespace adct
