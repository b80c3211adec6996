// The exact DCT-II as a comparison transform (Tables 1 and 2 compare the
// approximation against it) through Section 3.1's codec: per 16x16 block
// B = C A C^T, retention (zonal r x r or the first r of the zig-zag scan),
// X = C^T B C, output clamp(floor(X + 1/2)), with C the orthonormal DCT-II
// in fp32.
//
// The block products are dense 16x16x16 contractions, so they run on the
// matrix cores: v_mfma_f32_16x16x4_f32, four steps of K = 4 per product, one
// wave per block.  Operand layout of that instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] of one K-step, and receives
// D[4 (l / 16) + r][l % 16], r = 0..3.  The entries of C a lane needs are the
// same in every block and stay in registers; the block and the intermediate
// products pass between layouts through a 16 x 17 LDS array per wave.
#include <hip/hip_runtime.h>

#include <cmath>

#include "adct_internal.hpp"
#include "adct_tile.hpp"

namespace adct {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLd = 17;  // LDS row stride (floats)

struct DctArgs {
    const char* src;
    int64_t src_pitch;
    char* dst;
    int64_t dst_pitch;
    uint32_t nblk, bw, per_wave;  // blocks, blocks per block row, blocks per wave
    FastDiv bwdiv, ipbdiv;        // / bw, / block rows per image
    int32_t kind, r;              // retention: 0 zonal r x r, 1 first r of the zig-zag scan
    unsigned long long* sse;      // per image, or null
    float C[256];                 // C[k * 16 + j], orthonormal DCT-II in fp32
};

__device__ __forceinline__ void wave_sync() {
    // LDS writes of some lanes, reads of others, within one wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename S>
__global__ __launch_bounds__(256) void k_dct(DctArgs a) {
    __shared__ float buf[4][16 * kLd];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float* t = buf[wave];
    const int j16 = lane & 15, k4 = lane >> 4;   // MFMA operand coordinates
    const int row = lane >> 2, c0 = (lane & 3) * 4;  // sample coordinates: 4 per lane
    float cA[4], cB[4];  // cA[c] = C[j16][4c + k4], cB[c] = C[4c + k4][j16]
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        cA[c] = a.C[j16 * 16 + 4 * c + k4];
        cB[c] = a.C[(4 * c + k4) * 16 + j16];
    }
    constexpr int lo = sizeof(S) == 1 ? 0 : -255, hi = 255;
    const uint32_t w = blockIdx.x * 4u + (uint32_t)wave;
    const uint32_t first = w * a.per_wave, end = min(a.nblk, first + a.per_wave);
    long long acc = 0;
    uint32_t cur = 0xffffffffu;
    for (uint32_t g = first; g < end; ++g) {
        const uint32_t by = fdiv(g, a.bwdiv), bx = g - by * a.bw;
        const char* sp = a.src + (int64_t)(by * 16u + (uint32_t)row) * a.src_pitch + (int64_t)(bx * 16u + c0) * (int64_t)sizeof(S);
        int32_t x[4];
        if constexpr (sizeof(S) == 1) {
            const uint32_t v = *reinterpret_cast<const uint32_t*>(sp);
#pragma unroll
            for (int k = 0; k < 4; ++k) x[k] = (int32_t)((v >> (8 * k)) & 0xffu);
        } else {
            const uint2 v = *reinterpret_cast<const uint2*>(sp);
            x[0] = (int32_t)(int16_t)(v.x & 0xffffu);
            x[1] = (int32_t)(int16_t)(v.x >> 16);
            x[2] = (int32_t)(int16_t)(v.y & 0xffffu);
            x[3] = (int32_t)(int16_t)(v.y >> 16);
        }
        wave_sync();  // the previous block's reads of t are done
#pragma unroll
        for (int k = 0; k < 4; ++k) t[row * kLd + c0 + k] = (float)x[k];
        wave_sync();
        // P = X C^T
        f32x4 p = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) p = __builtin_amdgcn_mfma_f32_16x16x4f32(t[j16 * kLd + 4 * c + k4], cA[c], p, 0, 0, 0);
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * k4 + r) * kLd + j16] = p[r];
        wave_sync();
        // Y = C P, then retention
        f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) y = __builtin_amdgcn_mfma_f32_16x16x4f32(cA[c], t[(4 * c + k4) * kLd + j16], y, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int u = 4 * k4 + r, v = j16;
            const bool keep = a.kind == 0 ? (u < a.r && v < a.r) : (zigzag_rank(u, v) < a.r);
            if (!keep) y[r] = 0.f;
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * k4 + r) * kLd + j16] = y[r];
        wave_sync();
        // Q = Y C
        f32x4 q = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) q = __builtin_amdgcn_mfma_f32_16x16x4f32(t[j16 * kLd + 4 * c + k4], cB[c], q, 0, 0, 0);
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * k4 + r) * kLd + j16] = q[r];
        wave_sync();
        // X = C^T Q
        f32x4 o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) o = __builtin_amdgcn_mfma_f32_16x16x4f32(cB[c], t[(4 * c + k4) * kLd + j16], o, 0, 0, 0);
        wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) t[(4 * k4 + r) * kLd + j16] = o[r];
        wave_sync();
        // round half up and clamp the lane's four samples, store, SSE
        int32_t out[4];
        int32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float f = floorf(__fadd_rn(t[row * kLd + c0 + k], 0.5f));
            out[k] = (int32_t)fminf(fmaxf(f, (float)lo), (float)hi);
            const int32_t d = out[k] - x[k];
            s += d * d;
        }
        char* dp = a.dst + (int64_t)(by * 16u + (uint32_t)row) * a.dst_pitch + (int64_t)(bx * 16u + c0) * (int64_t)sizeof(S);
        if constexpr (sizeof(S) == 1) {
            *reinterpret_cast<uint32_t*>(dp) = (uint32_t)out[0] | ((uint32_t)out[1] << 8) | ((uint32_t)out[2] << 16) |
                                              ((uint32_t)out[3] << 24);
        } else {
            *reinterpret_cast<uint2*>(dp) = make_uint2(((uint32_t)out[0] & 0xffffu) | ((uint32_t)out[1] << 16),
                                                      ((uint32_t)out[2] & 0xffffu) | ((uint32_t)out[3] << 16));
        }
        if (a.sse) {
            // blocks of a wave run through images in order: one atomic per image
            const uint32_t img = fdiv(by, a.ipbdiv);
            if (img != cur) {
                long long v = acc;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0 && cur != 0xffffffffu && v) atomicAdd(a.sse + cur, (unsigned long long)v);
                acc = 0;
                cur = img;
            }
            acc += s;
        }
    }
    if (a.sse && cur != 0xffffffffu) {
        long long v = acc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0 && v) atomicAdd(a.sse + cur, (unsigned long long)v);
    }
}

__global__ __launch_bounds__(256) void k_dct_zero(unsigned long long* p, uint32_t n) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

}  // namespace

// Exact-DCT codec launch (argument checks done by the caller).
int launch_dct_codec(const adct_plane* src, int32_t kind, int r, const adct_plane* dst, int32_t image_height,
                     int64_t* sse, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    DctArgs a{};
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    a.dst = static_cast<char*>(dst->data);
    a.dst_pitch = dst->pitch_bytes;
    a.nblk = (uint32_t)((src->height / 16) * (src->width / 16));
    a.bw = (uint32_t)(src->width / 16);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(sse ? (uint32_t)(image_height / 16) : 1u);
    a.kind = kind;
    a.r = r;
    a.sse = reinterpret_cast<unsigned long long*>(sse);
    for (int k = 0; k < 16; ++k)
        for (int j = 0; j < 16; ++j) {
            const double al = k == 0 ? std::sqrt(1.0 / 16.0) : std::sqrt(2.0 / 16.0);
            a.C[k * 16 + j] = (float)(al * std::cos(M_PI * (2 * j + 1) * k / 32.0));
        }
    // about eight waves per CU's worth of blocks each, at least one block per wave
    const uint32_t waves = 256u * 32u;
    a.per_wave = (a.nblk + waves - 1) / waves;
    if (a.per_wave == 0) a.per_wave = 1;
    const uint32_t nwaves = (a.nblk + a.per_wave - 1) / a.per_wave;
    if (sse) {
        const uint32_t nimg = (uint32_t)(src->height / image_height);
        hipLaunchKernelGGL(k_dct_zero, dim3((nimg + 255) / 256), dim3(256), 0, s, a.sse, nimg);
        if (hipGetLastError() != hipSuccess) return ADCT_E_HIP;
    }
    if (a.nblk == 0) return ADCT_OK;
    const dim3 grid((nwaves + 3) / 4);
    if (src->dtype == ADCT_U8)
        hipLaunchKernelGGL(k_dct<uint8_t>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_dct<int16_t>, grid, dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP;
}

}  // namespace adct
