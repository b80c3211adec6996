// Image quality beside PSNR: the SSIM index (Wang, Bovik, Sheikh and
// Simoncelli, 2004) that Section 3.1 reports for the zig-zag experiment.
//
// Per image: local statistics under an 11x11 Gaussian window (standard
// deviation 1.5, unit sum) at every position where the window lies inside
// the image, SSIM at each such position, and their mean.  The window is
// separable.  A workgroup computes a tile of 16 x 48 positions from a
// 26 x 58 patch of both images (loaded as aligned 16-byte words):
//   horizontal pass: each thread takes one patch row and four adjacent
//     positions; the 14 samples they need are converted to float64 once
//     and their products formed once (exact), and the five weighted sums
//     (x, y, x^2, y^2, xy) take 11 multiply-adds per position, two
//     quantities' chains interleaved, and go to LDS;
//   vertical pass: each thread takes three positions of one column, reading
//     the 13 rows they need once per quantity.
// All of it is float64: the variances are differences of nearly equal
// moments.
#include <hip/hip_runtime.h>

#include <cmath>

#include "adct_internal.hpp"
#include "adct_tile.hpp"

namespace adct {
namespace {

constexpr int kWin = 11;                  // window side
constexpr int kTW = 16;                   // positions per tile row
#ifndef ADCT_SSIM_TH
#define ADCT_SSIM_TH 48
#endif
constexpr int kTH = ADCT_SSIM_TH;         // positions per tile column
constexpr int kPW = kTW + kWin - 1;       // 26: patch width
constexpr int kPH = kTH + kWin - 1;       // 58: patch height
constexpr int kHW = 4;                    // positions per thread, horizontal pass
constexpr int kVH = kTH / 16;             // positions per thread, vertical pass
constexpr int kLdh = kTW;                 // LDS row stride of the horizontal sums (doubles)
static_assert(kTH % 16 == 0 && (kTH / kVH) * kTW == 256, "one vertical work item per thread");
static_assert(kPW <= 32, "a patch row fits two 16-byte words");

struct SsimArgs {
    const uint8_t* a;
    const uint8_t* b;
    int64_t pitch_a, pitch_b;
    uint32_t width, image_height;
    uint32_t tiles_x, tiles_y;       // position tiles per image row / column
    uint32_t units;                  // images * tiles_y * tiles_x (below 2^31)
    FastDiv per_image_div, tiles_x_div;  // / (tiles_y * tiles_x), / tiles_x
    double w[kWin];                  // 1D Gaussian weights (outer product = window)
    double c1, c2;
    double* sum;                     // per image: sum of SSIM over positions
};

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// The 11-tap weighted sums of kHW adjacent positions over values v (one
// quantity), as kHW independent chains, written to out[0 .. kHW - 1].
template <int N>
__device__ __forceinline__ void taps1(const double (&w)[kWin], const double (&v)[N], double* out) {
    double acc[kHW];
#pragma unroll
    for (int m = 0; m < kHW; ++m) acc[m] = w[0] * v[m];
#pragma unroll
    for (int k = 1; k < kWin; ++k)
#pragma unroll
        for (int m = 0; m < kHW; ++m) acc[m] = fma(w[k], v[m + k], acc[m]);
#pragma unroll
    for (int m = 0; m < kHW; ++m) out[m] = acc[m];
}

// The same for two quantities at once (2 kHW chains).
template <int N>
__device__ __forceinline__ void taps2(const double (&w)[kWin], const double (&u)[N], const double (&v)[N],
                                      double* out_u, double* out_v) {
    double au[kHW], av[kHW];
#pragma unroll
    for (int m = 0; m < kHW; ++m) {
        au[m] = w[0] * u[m];
        av[m] = w[0] * v[m];
    }
#pragma unroll
    for (int k = 1; k < kWin; ++k)
#pragma unroll
        for (int m = 0; m < kHW; ++m) {
            au[m] = fma(w[k], u[m + k], au[m]);
            av[m] = fma(w[k], v[m + k], av[m]);
        }
#pragma unroll
    for (int m = 0; m < kHW; ++m) {
        out_u[m] = au[m];
        out_v[m] = av[m];
    }
}

// 40 KB of LDS and at most 128 VGPRs: four workgroups per CU.
__global__ __launch_bounds__(256) void k_ssim(SsimArgs s) {
    __shared__ uint4 pa[kPH][2], pb[kPH][2];  // patch rows as two 16-byte words (26 of 32 bytes used)
    __shared__ double h[5][kPH][kLdh];
    __shared__ double red[4];
    const int tid = threadIdx.x;
    const uint32_t per_image = s.tiles_x * s.tiles_y;
    const uint32_t valid_h = s.image_height - (kWin - 1), valid_w = s.width - (kWin - 1);
    for (uint32_t unit = blockIdx.x; unit < s.units; unit += gridDim.x) {
        // the tile's image and place: uniform, by multiply-high (no division
        // sequence on the vector unit)
        const uint32_t img = fdiv(unit, s.per_image_div), rem = unit - img * per_image;
        const uint32_t ty = fdiv(rem, s.tiles_x_div), tx = rem - ty * s.tiles_x;
        const uint32_t oy = ty * kTH, ox = tx * kTW;
        __syncthreads();  // the previous tile is done with LDS
        for (int t = tid; t < 4 * kPH; t += 256) {
            // one 16-byte word per step: row i, word k of image a or b.  ox
            // and the width are multiples of 16, so a word lies entirely
            // inside or outside the image; outside it feeds only positions
            // that are not used.
            const int i = t >> 2, k = t & 1, im = (t >> 1) & 1;
            const uint32_t y = oy + (uint32_t)i, x = ox + 16u * (uint32_t)k;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (y < s.image_height && x < s.width) {
                const int64_t row = (int64_t)img * s.image_height + y;
                v = im ? *reinterpret_cast<const uint4*>(s.b + row * s.pitch_b + x)
                       : *reinterpret_cast<const uint4*>(s.a + row * s.pitch_a + x);
            }
            (im ? pb : pa)[i][k] = v;
        }
        __syncthreads();
        for (int hw = tid; hw < kPH * (kTW / kHW); hw += 256) {
            // horizontal pass: patch row r, positions j0 .. j0 + 3
            const int r = hw / (kTW / kHW), j0 = (hw % (kTW / kHW)) * kHW;
            constexpr int kS = kHW + kWin - 1;
            double da[kS], db[kS];
            const uint8_t* ra = reinterpret_cast<const uint8_t*>(pa[r]);
            const uint8_t* rb = reinterpret_cast<const uint8_t*>(pb[r]);
#pragma unroll
            for (int c = 0; c < kS; ++c) {
                da[c] = (double)ra[j0 + c];
                db[c] = (double)rb[j0 + c];
            }
            double* out = &h[0][r][j0];
            constexpr int kQ = kPH * kLdh;  // LDS stride between the quantities (doubles)
            // x and y, then xy, then x^2 and y^2 (squared in place): eight or
            // four independent chains of 11 multiply-adds at a time
            taps2<kS>(s.w, da, db, out, out + kQ);
            {
                double p[kS];
#pragma unroll
                for (int c = 0; c < kS; ++c) p[c] = da[c] * db[c];
                taps1<kS>(s.w, p, out + 4 * kQ);
            }
#pragma unroll
            for (int c = 0; c < kS; ++c) {
                da[c] *= da[c];
                db[c] *= db[c];
            }
            taps2<kS>(s.w, da, db, out + 2 * kQ, out + 3 * kQ);
        }
        __syncthreads();
        // vertical pass: column j, positions i0 .. i0 + 2
        const int j = tid % kTW, i0 = (tid / kTW) * kVH;
        double st[5][kVH];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            double col[kVH + kWin - 1];
#pragma unroll
            for (int c = 0; c < kVH + kWin - 1; ++c) col[c] = h[q][i0 + c][j];
#pragma unroll
            for (int m = 0; m < kVH; ++m) {
                double v = s.w[0] * col[m];
#pragma unroll
                for (int k = 1; k < kWin; ++k) v = fma(s.w[k], col[m + k], v);
                // pinned here: the sums are formed now, so that this
                // quantity's column is dead before the next one is read
                // (otherwise every quantity's reads are hoisted ahead and
                // held in registers at once)
                __asm__ volatile("" : "+v"(v));
                st[q][m] = v;
            }
        }
        double v = 0.0;
#pragma unroll
        for (int m = 0; m < kVH; ++m) {
            if (oy + (uint32_t)(i0 + m) < valid_h && ox + (uint32_t)j < valid_w) {
                const double ma = st[0][m], mb = st[1][m];
                const double vaa = st[2][m] - ma * ma, vbb = st[3][m] - mb * mb, cab = st[4][m] - ma * mb;
                v += ((2.0 * ma * mb + s.c1) * (2.0 * cab + s.c2)) / ((ma * ma + mb * mb + s.c1) * (vaa + vbb + s.c2));
            }
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
    s.tiles_x = (vw + kTW - 1) / kTW;
    s.tiles_y = (vh + kTH - 1) / kTH;
    const uint64_t units = (uint64_t)nimg * s.tiles_x * s.tiles_y;
    if (units > (uint64_t)INT32_MAX) return ADCT_E_TOO_LARGE;
    s.units = (uint32_t)units;
    s.per_image_div = make_fastdiv(s.tiles_x * s.tiles_y);
    s.tiles_x_div = make_fastdiv(s.tiles_x);
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
    const uint32_t grid = s.units < 262144u ? s.units : 262144u;
    hipLaunchKernelGGL(k_ssim, dim3((unsigned)grid), dim3(256), 0, st, s);
    if ((rc = launched())) return rc;
    hipLaunchKernelGGL(k_scale_f64, dim3((nimg + 255) / 256), dim3(256), 0, st, ssim, nimg,
                       1.0 / ((double)vh * (double)vw));
    return launched();
}

}  // extern "C"
