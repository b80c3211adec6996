// Image quality beside PSNR: the SSIM index (Wang, Bovik, Sheikh and
// Simoncelli, 2004) that Section 3.1 reports for the zig-zag experiment.
//
// Per image: local statistics under an 11x11 Gaussian window (standard
// deviation 1.5, unit sum) at every position where the window lies inside
// the image, SSIM at each such position, and their mean.  The window is
// separable, so a workgroup computes a 16x16 tile of positions from a 26x26
// patch of both images: a horizontal pass (five weighted sums: x, y, x^2, y^2,
// xy) over 26 rows into LDS, then a vertical pass per position.  Everything
// is in float64: the variances are differences of nearly equal moments.
#include <hip/hip_runtime.h>

#include <cmath>

#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kWin = 11;             // window side
constexpr int kOut = 16;             // positions per tile side
constexpr int kPatch = kOut + kWin - 1;  // 26

struct SsimArgs {
    const uint8_t* a;
    const uint8_t* b;
    int64_t pitch_a, pitch_b;
    uint32_t width, image_height;
    uint32_t tiles_x, tiles_y;       // position tiles per image row / column
    uint64_t units;                  // images * tiles_y * tiles_x
    double w[kWin];                  // 1D Gaussian weights (outer product = window)
    double c1, c2;
    double* sum;                     // per image: sum of SSIM over positions
};

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_ssim(SsimArgs s) {
    __shared__ float pa[kPatch][kPatch + 1], pb[kPatch][kPatch + 1];
    __shared__ double h[5][kPatch][kOut];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const uint32_t per_image = s.tiles_x * s.tiles_y;
    const uint32_t valid_h = s.image_height - (kWin - 1), valid_w = s.width - (kWin - 1);
    for (uint64_t unit = blockIdx.x; unit < s.units; unit += gridDim.x) {
        const uint32_t img = (uint32_t)(unit / per_image), rem = (uint32_t)(unit % per_image);
        const uint32_t oy = (rem / s.tiles_x) * kOut, ox = (rem % s.tiles_x) * kOut;
        __syncthreads();  // the previous tile is done with LDS
        for (int t = tid; t < kPatch * kPatch; t += 256) {
            const int i = t / kPatch, j = t % kPatch;
            const uint32_t y = oy + (uint32_t)i, x = ox + (uint32_t)j;
            float va = 0.f, vb = 0.f;
            if (y < s.image_height && x < s.width) {  // outside: feeds only positions that are not used
                const int64_t row = (int64_t)img * s.image_height + y;
                va = (float)s.a[row * s.pitch_a + x];
                vb = (float)s.b[row * s.pitch_b + x];
            }
            pa[i][j] = va;
            pb[i][j] = vb;
        }
        __syncthreads();
        for (int t = tid; t < kPatch * kOut; t += 256) {
            const int i = t / kOut, j = t % kOut;
            double sa = 0, sb = 0, saa = 0, sbb = 0, sab = 0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double xa = pa[i][j + k], xb = pb[i][j + k], w = s.w[k];
                sa = fma(w, xa, sa);
                sb = fma(w, xb, sb);
                saa = fma(w, xa * xa, saa);
                sbb = fma(w, xb * xb, sbb);
                sab = fma(w, xa * xb, sab);
            }
            h[0][i][j] = sa;
            h[1][i][j] = sb;
            h[2][i][j] = saa;
            h[3][i][j] = sbb;
            h[4][i][j] = sab;
        }
        __syncthreads();
        const int i = tid / kOut, j = tid % kOut;
        double v = 0.0;
        if (oy + (uint32_t)i < valid_h && ox + (uint32_t)j < valid_w) {
            double ma = 0, mb = 0, eaa = 0, ebb = 0, eab = 0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double w = s.w[k];
                ma = fma(w, h[0][i + k][j], ma);
                mb = fma(w, h[1][i + k][j], mb);
                eaa = fma(w, h[2][i + k][j], eaa);
                ebb = fma(w, h[3][i + k][j], ebb);
                eab = fma(w, h[4][i + k][j], eab);
            }
            const double vaa = eaa - ma * ma, vbb = ebb - mb * mb, cab = eab - ma * mb;
            v = ((2.0 * ma * mb + s.c1) * (2.0 * cab + s.c2)) / ((ma * ma + mb * mb + s.c1) * (vaa + vbb + s.c2));
        }
        v = wave_sum_f64(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) atomicAdd(s.sum + img, red[0] + red[1] + red[2] + red[3]);
    }
}

__global__ __launch_bounds__(256) void k_fill_f64(double* p, uint32_t n, double v) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ __launch_bounds__(256) void k_scale_f64(double* p, uint32_t n, double f) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] *= f;
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

int adct_ssim(const adct_plane* a, const adct_plane* b, int32_t image_height, double* ssim, void* stream) {
    int rc = check_plane(a);
    if (rc) return rc;
    if ((rc = check_plane(b))) return rc;
    if (a->dtype != ADCT_U8) return ADCT_E_DTYPE;
    if (!same_shape(a, b)) return ADCT_E_SHAPE;
    if (!ssim) return ADCT_E_ARG;
    if (((uintptr_t)ssim) & 7) return ADCT_E_ALIGN;
    if (image_height <= 0 || (image_height & 15) || a->height % image_height) return ADCT_E_SHAPE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t nimg = (uint32_t)(a->height / image_height);
    SsimArgs s{};
    s.a = static_cast<const uint8_t*>(a->data);
    s.b = static_cast<const uint8_t*>(b->data);
    s.pitch_a = a->pitch_bytes;
    s.pitch_b = b->pitch_bytes;
    s.width = (uint32_t)a->width;
    s.image_height = (uint32_t)image_height;
    const uint32_t vh = s.image_height - (kWin - 1), vw = s.width - (kWin - 1);
    s.tiles_x = (vw + kOut - 1) / kOut;
    s.tiles_y = (vh + kOut - 1) / kOut;
    s.units = (uint64_t)nimg * s.tiles_x * s.tiles_y;
    double g[kWin], gs = 0.0;
    for (int k = 0; k < kWin; ++k) {
        const double d = k - (kWin - 1) / 2.0;
        g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        gs += g[k];
    }
    for (int k = 0; k < kWin; ++k) s.w[k] = g[k] / gs;
    s.c1 = (0.01 * 255.0) * (0.01 * 255.0);
    s.c2 = (0.03 * 255.0) * (0.03 * 255.0);
    s.sum = ssim;
    hipLaunchKernelGGL(k_fill_f64, dim3((nimg + 255) / 256), dim3(256), 0, st, ssim, nimg, 0.0);
    if ((rc = launched())) return rc;
    const uint64_t grid = s.units < 262144 ? s.units : 262144;
    hipLaunchKernelGGL(k_ssim, dim3((unsigned)grid), dim3(256), 0, st, s);
    if ((rc = launched())) return rc;
    hipLaunchKernelGGL(k_scale_f64, dim3((nimg + 255) / 256), dim3(256), 0, st, ssim, nimg,
                       1.0 / ((double)vh * (double)vw));
    return launched();
}

}  // extern "C"
