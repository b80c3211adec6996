// The 8-point approximation T8 on 8x8 blocks (the 8-point half of the
// paper's second video scenario, Section 3.2).  T8's butterflies (14
// additions) and quantiser factors are in adct_t8_common.hpp.
//
// One thread owns one 8x8 block, entirely in registers: the row pass, the
// column pass, the retention or quantisation step, both inverse passes and
// the rounding all run without LDS.  Consecutive lanes own consecutive
// blocks of a block row, so each of the eight row loads (8 bytes per lane
// for uint8, 16 for int16) and stores is one contiguous run per wave.
// Coefficient blocks (256 bytes int32 or 128 bytes int16 per block) are
// staged through LDS by the wave and written as contiguous runs.
//
// Fixed point: with d = diag(T8 T8^T) = (8,2,4,2,8,2,4,2), the weights
// W8 = 64 / (d_u d_v) (a shift of 0..5 bits) make T8^T (W8 . T8 X T8^T) T8
// = 64 X exact, so reconstructions carry 6 fractional bits and are rounded
// as floor((R + 32) / 64).
#include <hip/hip_runtime.h>

#include <cmath>

#include "adct_internal.hpp"
#include "adct_t8_common.hpp"
#include "adct_tile.hpp"
#include "adct_zero.hpp"

namespace adct {
namespace {

enum Op8 { kFwd8 = 0, kZonal8 = 1, kQuant8 = 2 };

struct Args8 {
    const char* src;
    int64_t src_pitch;
    char* dst;
    int64_t dst_pitch;
    void* cout;              // int32 Y (zonal, forward) or int16 q (quant); null: not stored
    uint32_t nblk, bw;       // blocks, blocks per block row
    FastDiv bwdiv, ipbdiv;   // / bw, / block rows per image
    int32_t r;               // zonal size
    float qs[5], dqs[5];     // per class c = log2 d_u + log2 d_v - 2
    unsigned long long* sse; // per image, or null
    uint32_t spread_rows;    // 0: workgroup b takes chunk b; else see k_t8
};

// Workgroups of a launch that adds to the SSE of large images are dealt
// over the plane in this many interleaved streams (as the 16-point group
// kernel does), so that the workgroups resident at one time add to several
// images' sums instead of queueing on the atomics of one, while each stream
// stays a sequential sweep of its part of the plane.
constexpr uint32_t kSpread8 = 4;
constexpr uint32_t kSpreadMin8 = 16;  // chunks of 256 blocks per image

// One block row as raw words (uint8: 8 samples in w.x, w.y; int16: 8
// samples in w.x .. w.w), and the same unpacked to int32.
template <typename S>
__device__ __forceinline__ uint4 load_row8(const char* p) {
    if constexpr (sizeof(S) == 1) {
        const uint2 w = *reinterpret_cast<const uint2*>(p);
        return make_uint4(w.x, w.y, 0u, 0u);
    } else {
        return *reinterpret_cast<const uint4*>(p);
    }
}

template <typename S>
__device__ __forceinline__ void unpack_row8(const uint4& w, int32_t (&v)[8]) {
    if constexpr (sizeof(S) == 1) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = (int32_t)((w.x >> (8 * j)) & 0xffu);
            v[4 + j] = (int32_t)((w.y >> (8 * j)) & 0xffu);
        }
    } else {
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[2 * j] = (int32_t)(int16_t)(ws[j] & 0xffffu);
            v[2 * j + 1] = (int32_t)(int16_t)(ws[j] >> 16);
        }
    }
}

template <typename S>
__device__ __forceinline__ void store_row8(char* p, const int32_t (&v)[8]) {
    if constexpr (sizeof(S) == 1) {
        uint2 w;
        w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
        w.y = (uint32_t)v[4] | ((uint32_t)v[5] << 8) | ((uint32_t)v[6] << 16) | ((uint32_t)v[7] << 24);
        *reinterpret_cast<uint2*>(p) = w;
    } else {
        uint4 w;
        w.x = ((uint32_t)v[0] & 0xffffu) | ((uint32_t)v[1] << 16);
        w.y = ((uint32_t)v[2] & 0xffffu) | ((uint32_t)v[3] << 16);
        w.z = ((uint32_t)v[4] & 0xffffu) | ((uint32_t)v[5] << 16);
        w.w = ((uint32_t)v[6] & 0xffffu) | ((uint32_t)v[7] << 16);
        *reinterpret_cast<uint4*>(p) = w;
    }
}

__device__ __forceinline__ float pick8(const float (&t)[5], int c) {
    float r = t[4];
    r = (c == 3) ? t[3] : r;
    r = (c == 2) ? t[2] : r;
    r = (c == 1) ? t[1] : r;
    r = (c == 0) ? t[0] : r;
    return r;
}

// Each wave writes its 64 blocks' coefficients (block-major, so one
// contiguous run) through LDS, half a block (HALF 32-bit words) at a time:
// lane L's words go to row L of a padded 64 x (HALF + 1) array, then the
// wave stores the halves as 16-byte pieces, each half a contiguous run of
// HALF * 4 bytes inside its block.  Called by every thread of the
// workgroup (it holds workgroup barriers).
template <int HALF>
__device__ __forceinline__ void wave_store_half(uint32_t* lds, const uint32_t (&w)[HALF], char* out_wave,
                                                int half, uint32_t nvalid) {
    const int lane = threadIdx.x & 63;
    __syncthreads();  // earlier readers of this LDS slice are done
#pragma unroll
    for (int i = 0; i < HALF; ++i) lds[lane * (HALF + 1) + i] = w[i];
    __syncthreads();
    constexpr int kPieces = HALF / 4;  // 16-byte pieces per half block
#pragma unroll
    for (int k = 0; k < kPieces; ++k) {
        const int piece = k * 64 + lane;
        const int blk = piece / kPieces, part = piece % kPieces;
        if ((uint32_t)blk < nvalid) {
            const uint32_t* src = lds + blk * (HALF + 1) + part * 4;
            const uint4 v = make_uint4(src[0], src[1], src[2], src[3]);
            *reinterpret_cast<uint4*>(out_wave + (int64_t)blk * (2 * HALF * 4) + half * (HALF * 4) + part * 16) = v;
        }
    }
}

// Workgroup b of a launch over the plane of `a` (256 threads).
template <typename S, int OP, bool STORE, bool SSE>
__device__ __forceinline__ void t8_chunk(const Args8& a, uint32_t b) {
    constexpr int kHalf = OP == kQuant8 ? 16 : 32;  // 32-bit words of half a stored block
    __shared__ uint32_t lds[4][64 * (kHalf + 1)];
    __shared__ long long red[2][4];
    // the block's input rows, kept for the SSE: row i of thread t at
    // src_rows[i][t] (consecutive threads, consecutive words: no conflicts)
    constexpr int kRowWords = sizeof(S) == 1 ? 2 : 4;
    __shared__ uint32_t src_rows[SSE ? 8 : 1][SSE ? 256 * kRowWords : 1];
    // chunk of 256 consecutive blocks taken by this workgroup
    const uint32_t chunk = a.spread_rows ? (b % kSpread8) * a.spread_rows + b / kSpread8 : b;
    const uint32_t first = chunk * 256u;
    if (first >= a.nblk) return;  // past the last chunk (spread grids only)
    const uint32_t g = first + threadIdx.x;
    const bool ok = g < a.nblk;
    const uint32_t gs = ok ? g : a.nblk - 1;
    const uint32_t by = fdiv(gs, a.bwdiv), bx = gs - by * a.bw;
    uint4 raw[8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
        raw[i] = load_row8<S>(a.src + (int64_t)(by * 8u + (uint32_t)i) * a.src_pitch + (int64_t)bx * 8 * (int64_t)sizeof(S));
    if constexpr (SSE) {
        // the source rows leave L2 long before the SSE needs them again:
        // keep them in LDS (each thread reads back only its own rows)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint32_t* d = &src_rows[i][threadIdx.x * kRowWords];
            d[0] = raw[i].x;
            d[1] = raw[i].y;
            if constexpr (kRowWords == 4) {
                d[2] = raw[i].z;
                d[3] = raw[i].w;
            }
        }
    }
    // forward: rows, then columns
    int32_t y[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int32_t x[8];
        unpack_row8<S>(raw[i], x);
        fwd8(x, y[i]);
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        int32_t c[8], o[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] = y[u][v];
        fwd8(c, o);
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u][v] = o[u];
    }
    const int wave = threadIdx.x >> 6;
    const uint32_t wave_first = first + (uint32_t)wave * 64u;
    const uint32_t nvalid = a.nblk > wave_first ? min(64u, a.nblk - wave_first) : 0u;
    if constexpr (OP == kQuant8) {
        // the levels fit int16 without saturation: |Y| <= d_u d_v * 2047 for
        // samples within [-2047, 2047] (uint8: 255), so |Y s_u s_v| <=
        // sqrt(d_u d_v) * 2047 <= 16376 and 1 / Delta < 1.6 keep every level
        // below 26000 at any QP
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int v = 0; v < 8; ++v)
                y[u][v] = round_away(__fmul_rn((float)y[u][v], pick8(a.qs, l8(u) + l8(v) - 2)));
    }
    if constexpr (STORE) {
        if (a.cout) {
            char* out = static_cast<char*>(a.cout) + (int64_t)wave_first * (2 * kHalf * 4);
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                uint32_t w[kHalf];
                if constexpr (OP == kQuant8) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int e = half * 32 + 2 * i;  // element u * 8 + v
                        w[i] = ((uint32_t)y[e / 8][e % 8] & 0xffffu) | ((uint32_t)y[(e + 1) / 8][(e + 1) % 8] << 16);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < 32; ++i) w[i] = (uint32_t)y[(half * 32 + i) / 8][(half * 32 + i) % 8];
                }
                wave_store_half<kHalf>(lds[wave], w, out, half, nvalid);
            }
        }
    }
    if constexpr (OP == kFwd8) return;
    // the second half starts here: nothing of it (the reloads of the source
    // rows in particular) is scheduled into the forward half
    __builtin_amdgcn_sched_barrier(0);
    // retention or dequantisation, into 6 fractional bits
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            if constexpr (OP == kZonal8) {
                const bool keep = u < a.r && v < a.r;
                y[u][v] = keep ? (int32_t)((uint32_t)y[u][v] << (6 - l8(u) - l8(v))) : 0;
            } else {
                y[u][v] = round_away(__fmul_rn((float)y[u][v], pick8(a.dqs, l8(u) + l8(v) - 2)));
            }
        }
    y[0][0] += 32;  // rounding offset: DC reaches every sample with weight 1
    // inverse: columns, then rows
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        int32_t c[8], o[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] = y[u][v];
        inv8(c, o);
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u][v] = o[u];
    }
    constexpr int32_t lo = sizeof(S) == 1 ? 0 : -255, hi = 255;
    int32_t sse = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int32_t row[8], x[8];
        inv8(y[i], row);
        if constexpr (SSE) {
            // the source row from LDS rather than live registers through the
            // whole computation
            const uint32_t* d = &src_rows[i][threadIdx.x * kRowWords];
            unpack_row8<S>(kRowWords == 4 ? make_uint4(d[0], d[1], d[2], d[3]) : make_uint4(d[0], d[1], 0u, 0u), x);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // clamp before the shift (floor((R + 32) / 64) lands in [lo, hi])
            const int32_t o = clamp_i32(row[j], lo * 64, hi * 64 + 63) >> 6;
            row[j] = o;
            const int32_t d = o - x[j];
            sse += d * d;
        }
        if (ok) store_row8<S>(a.dst + (int64_t)(by * 8u + (uint32_t)i) * a.dst_pitch + (int64_t)bx * 8 * (int64_t)sizeof(S),
                              row);
    }
    if constexpr (SSE) {
        if (!ok) sse = 0;
        // the blocks of one workgroup lie in at most two images unless the
        // images are smaller than a workgroup's 256 blocks
        const uint32_t last = min(a.nblk, first + 256u) - 1u;
        const uint32_t img0 = fdiv(fdiv(first, a.bwdiv), a.ipbdiv), img1 = fdiv(fdiv(last, a.bwdiv), a.ipbdiv);
        if (img1 - img0 <= 1u) {
            const bool in0 = !ok || fdiv(by, a.ipbdiv) == img0;
            long long v0 = in0 ? sse : 0, v1 = in0 ? 0 : sse;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                v0 += __shfl_xor(v0, off, 64);
                v1 += __shfl_xor(v1, off, 64);
            }
            if ((threadIdx.x & 63) == 0) {
                red[0][wave] = v0;
                red[1][wave] = v1;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                const long long t0 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
                const long long t1 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
                if (t0) atomicAdd(a.sse + img0, (unsigned long long)t0);
                if (t1) atomicAdd(a.sse + img1, (unsigned long long)t1);
            }
        } else if (ok && sse) {
            atomicAdd(a.sse + fdiv(by, a.ipbdiv), (unsigned long long)sse);
        }
    }
}

template <typename S, int OP, bool STORE, bool SSE>
__global__ __launch_bounds__(256) void k_t8(Args8 a) {
    t8_chunk<S, OP, STORE, SSE>(a, blockIdx.x);
}

// Several planes in one launch: plane i takes the workgroups from first[i]
// (ascending) up to the next plane's, as k_t8 would over that plane alone.
struct Set8 {
    Args8 p[ADCT_MAX_PLANES];
    uint32_t first[ADCT_MAX_PLANES];
    uint32_t n;
};

template <typename S, int OP, bool STORE, bool SSE>
__global__ __launch_bounds__(256) void k_t8_planes(Set8 ps) {
    uint32_t i = 0;
#pragma unroll
    for (uint32_t k = 1; k < (uint32_t)ADCT_MAX_PLANES; ++k)
        if (k < ps.n && blockIdx.x >= ps.first[k]) i = k;
    t8_chunk<S, OP, STORE, SSE>(ps.p[i], blockIdx.x - ps.first[i]);
}

// T8^T Y T8 per block (block-major int32 in and out).
__global__ __launch_bounds__(256) void k_t8_inv(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                               uint32_t nblk) {
    const uint32_t g = blockIdx.x * 256u + threadIdx.x;
    if (g >= nblk) return;
    int32_t y[8][8];
    const int4* p = reinterpret_cast<const int4*>(in + (int64_t)g * 64);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int4 v = p[k];
        y[k / 2][(k % 2) * 4 + 0] = v.x;
        y[k / 2][(k % 2) * 4 + 1] = v.y;
        y[k / 2][(k % 2) * 4 + 2] = v.z;
        y[k / 2][(k % 2) * 4 + 3] = v.w;
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        int32_t c[8], o[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) c[u] = y[u][v];
        inv8(c, o);
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u][v] = o[u];
    }
    int4* q = reinterpret_cast<int4*>(out + (int64_t)g * 64);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        int32_t row[8];
        inv8(y[i], row);
        q[2 * i] = make_int4(row[0], row[1], row[2], row[3]);
        q[2 * i + 1] = make_int4(row[4], row[5], row[6], row[7]);
    }
}

__global__ __launch_bounds__(256) void k_t8_zero(unsigned long long* p, uint32_t n) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

// Planes of the 8-point calls: sides multiples of 8; rows aligned to one
// block row (8 bytes for uint8, 16 for int16), the width of the row loads.
int check_plane8(const adct_plane* p) {
    if (!p || !p->data) return ADCT_E_ARG;
    const int sz = sample_bytes(p->dtype);
    if (!sz) return ADCT_E_DTYPE;
    if (p->height <= 0 || p->width <= 0 || (p->height & 7) || (p->width & 7)) return ADCT_E_SHAPE;
    if (p->pitch_bytes < (int64_t)p->width * sz) return ADCT_E_SHAPE;
    const int64_t row_align = 8 * sz;
    if ((p->pitch_bytes % row_align) || (((uintptr_t)p->data) % row_align)) return ADCT_E_ALIGN;
    if ((int64_t)(p->height / 8) * (p->width / 8) > (int64_t)INT32_MAX - 256) return ADCT_E_SHAPE;
    return ADCT_OK;
}

int64_t blocks8(const adct_plane* p) { return (int64_t)(p->height / 8) * (p->width / 8); }

uint32_t grid8(const Args8& a) { return a.spread_rows ? a.spread_rows * kSpread8 : (a.nblk + 255) / 256; }

template <typename S, int OP, bool STORE>
void launch8(const Args8& a, hipStream_t s) {
    const dim3 grid(grid8(a));
    if (a.sse)
        hipLaunchKernelGGL((k_t8<S, OP, STORE, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_t8<S, OP, STORE, false>), grid, dim3(256), 0, s, a);
}

template <int OP>
int launch8_typed(int32_t dtype, const Args8& a, hipStream_t s) {
    if (a.nblk == 0) return ADCT_OK;
    if (dtype == ADCT_U8) {
        if (a.cout) launch8<uint8_t, OP, true>(a, s); else launch8<uint8_t, OP, false>(a, s);
    } else {
        if (a.cout) launch8<int16_t, OP, true>(a, s); else launch8<int16_t, OP, false>(a, s);
    }
    return launched();
}

// Shared checks and set-up of the encoders' arguments (no launch).
int setup_args8(const adct_plane* src, void* coef, const adct_plane* dst, int32_t image_height, int64_t* sse,
                Args8& a) {
    int rc = check_plane8(src);
    if (rc) return rc;
    if ((rc = check_plane8(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (sse && (image_height <= 0 || (image_height & 7) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    if (coef && (((uintptr_t)coef) & 15)) return ADCT_E_ALIGN;
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    a.dst = static_cast<char*>(dst->data);
    a.dst_pitch = dst->pitch_bytes;
    a.cout = coef;
    a.nblk = (uint32_t)blocks8(src);
    a.bw = (uint32_t)(src->width / 8);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(sse ? (uint32_t)(image_height / 8) : 1u);
    a.sse = reinterpret_cast<unsigned long long*>(sse);
    if (sse) {
        const uint32_t chunks = (a.nblk + 255) / 256;
        const uint32_t image_blocks = (uint32_t)(image_height / 8) * a.bw;
        if (image_blocks / 256 > kSpreadMin8) a.spread_rows = (chunks + kSpread8 - 1) / kSpread8;
    }
    return ADCT_OK;
}

// Checks, argument set-up and the clear of the SSE outputs of one encoder call.
int setup_encoder(const adct_plane* src, void* coef, const adct_plane* dst, int32_t image_height, int64_t* sse,
                  hipStream_t s, Args8& a) {
    const int rc = setup_args8(src, coef, dst, image_height, sse, a);
    if (rc || !sse) return rc;
    const uint32_t nimg = (uint32_t)(src->height / image_height);
    hipLaunchKernelGGL(k_t8_zero, dim3((nimg + 255) / 256), dim3(256), 0, s, a.sse, nimg);
    return launched();
}

template <typename S, bool STORE, bool SSE>
void launch8_planes(const Set8& ps, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL((k_t8_planes<S, kQuant8, STORE, SSE>), dim3(grid), dim3(256), 0, s, ps);
}

template <typename S>
void launch8_planes_typed(const Set8& ps, uint32_t grid, bool store, bool sse, hipStream_t s) {
    if (store) {
        if (sse) launch8_planes<S, true, true>(ps, grid, s); else launch8_planes<S, true, false>(ps, grid, s);
    } else {
        if (sse) launch8_planes<S, false, true>(ps, grid, s); else launch8_planes<S, false, false>(ps, grid, s);
    }
}

}  // namespace

int t8_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, void* stream) {
    float qs[5], dqs[5];
    if (!quant_scales8(qp, qs, dqs)) return ADCT_E_ARG;
    const bool store = jobs[0].q != nullptr, want_sse = jobs[0].sse != nullptr;
    const int32_t dt = jobs[0].src.dtype;
    Set8 ps{};
    ZeroSet<ADCT_MAX_PLANES> zs{};
    uint64_t grid = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        const adct_quant_job& j = jobs[i];
        if (j.src.dtype != dt || (j.q != nullptr) != store || (j.sse != nullptr) != want_sse) return ADCT_E_ARG;
        Args8& a = ps.p[i];
        const int rc = setup_args8(&j.src, j.q, &j.dst, j.image_height, j.sse, a);
        if (rc) return rc;
        for (int c = 0; c < 5; ++c) {
            a.qs[c] = qs[c];
            a.dqs[c] = dqs[c];
        }
        ps.first[i] = (uint32_t)grid;
        grid += grid8(a);
        if (want_sse) {
            zs.p[i] = a.sse;
            zs.n[i] = (uint32_t)(j.src.height / j.image_height);
        }
    }
    if (grid > (uint64_t)INT32_MAX) return ADCT_E_TOO_LARGE;
    ps.n = (uint32_t)njobs;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (want_sse) {
        zs.count = (uint32_t)njobs;
        clear_sets(zs, s);
    }
    if (dt == ADCT_U8)
        launch8_planes_typed<uint8_t>(ps, (uint32_t)grid, store, want_sse, s);
    else
        launch8_planes_typed<int16_t>(ps, (uint32_t)grid, store, want_sse, s);
    return launched();
}

}  // namespace adct

using namespace adct;

extern "C" {

int adct_t8_constants(int32_t* T64, double* s8, int32_t* W64) {
    static const int32_t kT8[8][8] = {
        {1, 1, 1, 1, 1, 1, 1, 1},   {1, 0, 0, 0, 0, 0, 0, -1},  {1, 0, 0, -1, -1, 0, 0, 1},
        {0, 0, -1, 0, 0, 1, 0, 0},  {1, -1, -1, 1, 1, -1, -1, 1}, {0, -1, 0, 0, 0, 0, 1, 0},
        {0, -1, 1, 0, 0, 1, -1, 0}, {0, 0, 0, -1, 1, 0, 0, 0}};
    for (int u = 0; u < 8; ++u) {
        if (T64)
            for (int j = 0; j < 8; ++j) T64[u * 8 + j] = kT8[u][j];
        if (s8) s8[u] = 1.0 / std::sqrt((double)(1 << l8(u)));
        if (W64)
            for (int v = 0; v < 8; ++v) W64[u * 8 + v] = 64 >> (l8(u) + l8(v));
    }
    return ADCT_OK;
}

int adct_t8_quant_tables(int qp, float* qs64, float* dqs64) {
    float qs[5], dqs[5];
    if (!quant_scales8(qp, qs, dqs)) return ADCT_E_ARG;
    for (int u = 0; u < 8; ++u)
        for (int v = 0; v < 8; ++v) {
            const int c = l8(u) + l8(v) - 2;
            if (qs64) qs64[u * 8 + v] = qs[c];
            if (dqs64) dqs64[u * 8 + v] = dqs[c];
        }
    return ADCT_OK;
}

int adct_t8_fwd2d(const adct_plane* src, int32_t* coef, void* stream) {
    int rc = check_plane8(src);
    if (rc) return rc;
    if (!coef) return ADCT_E_ARG;
    if (((uintptr_t)coef) & 15) return ADCT_E_ALIGN;
    Args8 a{};
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    a.cout = coef;
    a.nblk = (uint32_t)blocks8(src);
    a.bw = (uint32_t)(src->width / 8);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(1);
    return launch8_typed<kFwd8>(src->dtype, a, static_cast<hipStream_t>(stream));
}

int adct_t8_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream) {
    if (nblk < 0 || nblk > (int64_t)INT32_MAX - 256) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;  // an empty array may be a null pointer
    if (!coef || !out) return ADCT_E_ARG;
    if ((((uintptr_t)coef) & 15) || (((uintptr_t)out) & 15)) return ADCT_E_ALIGN;
    hipLaunchKernelGGL(k_t8_inv, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       coef, out, (uint32_t)nblk);
    return launched();
}

int adct_t8_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst, int32_t image_height,
                       int64_t* sse, void* stream) {
    if (r < 0 || r > 8) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args8 a{};
    int rc = setup_encoder(src, coef, dst, image_height, sse, s, a);
    if (rc) return rc;
    a.r = r;
    return launch8_typed<kZonal8>(src->dtype, a, s);
}

int adct_t8_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst, int32_t image_height,
                       int64_t* sse, void* stream) {
    float qs[5], dqs[5];
    if (!quant_scales8(qp, qs, dqs)) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args8 a{};
    int rc = setup_encoder(src, q, dst, image_height, sse, s, a);
    if (rc) return rc;
    for (int c = 0; c < 5; ++c) {
        a.qs[c] = qs[c];
        a.dqs[c] = dqs[c];
    }
    return launch8_typed<kQuant8>(src->dtype, a, s);
}

}  // extern "C"
