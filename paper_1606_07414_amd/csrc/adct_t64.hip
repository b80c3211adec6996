// The 64x64 codec of the 64-point extension T64 (butterflies in
// adct_t64_common.hpp): forward transform, zonal retention or quantisation
// with S folded in, inverse, rounding and the per-image SSE, one pass.
//
// A workgroup of 128 threads codes 2 consecutive tiles (raster order).
//   row role     rt = tid % 2, rr = tid / 2: row rr of tile rt, so the 2
//                lanes of one sample row read 2 horizontally adjacent
//                64-sample segments (contiguous for tiles of one tile row)
//   column role  ct = tid / 64, cv = tid % 64: column cv of tile ct, one
//                wave per tile, so a wave's lanes touch 64 adjacent
//                coefficients of one row of a block (256 contiguous bytes
//                of int32)
// The row pass runs in registers and goes to LDS ([tile][row][65 words],
// tile stride 4168 words: both roles' accesses are free of bank
// conflicts); the column pass, the coefficient domain and the inverse
// column pass run in the column role; the inverse row pass in the row role
// again after a second LDS transpose.  Two tiles take 33 KB of LDS, so a
// CU holds 4 workgroups (8 waves); each thread keeps whole 64-value rows
// and columns in registers, which that occupancy leaves room for.
//
// Fixed point: the weights 4096 / (d_u d_v) make T64^T (W . T64 X T64^T) T64
// = 4096 X exact; reconstructions are rounded as floor((R + 2048) / 4096).
// Every intermediate fits int32 for int16 samples within [-2047, 2047]:
// |Y| <= 64 * 64 * 2047 < 2^24, and the inverse of dequantised levels
// stays within 4096 |X| plus the quantisation error's transform.
#include <hip/hip_runtime.h>

#include "adct_core.hpp"
#include "adct_internal.hpp"
#include "adct_round.hpp"
#include "adct_t64_common.hpp"
#include "adct_tile.hpp"

namespace adct {
namespace {

enum Op64 { kFwd64 = 0, kZonal64 = 1, kQuant64 = 2 };

struct Args64 {
    const char* src;
    int64_t src_pitch;
    char* dst;
    int64_t dst_pitch;
    void* cout;              // int32 Y (forward, zonal) or int16 levels (quant); null: not stored
    uint32_t nblk, bw;       // tiles, tiles per tile row
    FastDiv bwdiv, ipbdiv;   // / bw, / tile rows per image
    int32_t r;               // zonal size
    Scale5 qs, dqs;          // per class c = log2 d_u + log2 d_v - 8
    unsigned long long* sse; // per image, or null
    uint32_t spread_rows;    // 0: workgroup b takes group b; else interleaved (see t64_group)
    bool sat;                // quantising: levels may leave int16 and are saturated (host side)
};

// Whether the levels of a 64x64 quantising call can leave int16.  A level is
// at most sqrt(d_u d_v) |x|max / Delta <= 64 |x|max / Delta (entries of T64
// in {0, +1, -1}, d_u of them nonzero in row u): for uint8 samples 16320 /
// Delta, within int16 at every QP (Delta >= 0.63); for int16 samples within
// +-2047 it is 131008 / Delta, within int16 from QP 16 (Delta = 4) on.
bool levels_may_saturate64(int32_t dtype, int qp) { return dtype != ADCT_U8 && qp < 16; }

constexpr int kTiles64 = 2;                 // tiles per workgroup
constexpr int kThreads64 = 64 * kTiles64;   // threads per workgroup
constexpr int kRow64 = 65;                  // LDS words per staged row
constexpr int kTile64 = 64 * kRow64 + 8;    // LDS words per staged tile
// Workgroups of a launch that adds to the SSE of large images are dealt
// over the plane in this many interleaved streams (as the 16-point group
// kernel does), so that the workgroups resident at one time add to several
// images' sums instead of queueing on the atomics of one, while each stream
// stays a sequential sweep of its part of the plane.
constexpr uint32_t kSpread64 = 4;
constexpr uint32_t kSpreadMin64 = 16;       // groups of 2 tiles per image

// Raw words of one 64-sample row (uint8: 16 words, int16: 32).
template <typename S>
struct Row64 {
    static constexpr int kWords = 16 * (int)sizeof(S);
    uint32_t w[kWords];
};

template <typename S>
__device__ __forceinline__ void load_row64(const char* p, Row64<S>& r) {
#pragma unroll
    for (int k = 0; k < Row64<S>::kWords / 4; ++k) {
        const uint4 v = reinterpret_cast<const uint4*>(p)[k];
        r.w[4 * k] = v.x;
        r.w[4 * k + 1] = v.y;
        r.w[4 * k + 2] = v.z;
        r.w[4 * k + 3] = v.w;
    }
}

template <typename S>
__device__ __forceinline__ int32_t sample64(const Row64<S>& r, int j) {
    if constexpr (sizeof(S) == 1)
        return (int32_t)((r.w[j >> 2] >> (8 * (j & 3))) & 0xffu);
    else
        return (j & 1) ? ((int32_t)r.w[j >> 1] >> 16) : (int32_t)(int16_t)(r.w[j >> 1] & 0xffffu);
}

// The 64 output samples of a row as raw words, the layout of Row64.
template <typename S>
__device__ __forceinline__ void pack_row64(const int32_t (&o)[64], uint32_t (&w)[Row64<S>::kWords]) {
    if constexpr (sizeof(S) == 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            w[i] = (uint32_t)o[4 * i] | ((uint32_t)o[4 * i + 1] << 8) | ((uint32_t)o[4 * i + 2] << 16) |
                   ((uint32_t)o[4 * i + 3] << 24);
    } else {
#pragma unroll
        for (int i = 0; i < 32; ++i) w[i] = ((uint32_t)o[2 * i] & 0xffffu) | ((uint32_t)o[2 * i + 1] << 16);
    }
}

// Output rows leave through LDS: each thread stages its packed row, then the
// workgroup stores 16-byte chunks with consecutive threads on consecutive
// chunks of a sample row (both tiles' segments of that row in turn), so
// every store instruction writes whole contiguous lines.
template <typename S>
__device__ __forceinline__ void store_rows64(int32_t* lds, const uint32_t (&w)[Row64<S>::kWords], const Args64& a,
                                             uint32_t g0, uint32_t ntile) {
    constexpr int kW = Row64<S>::kWords;  // words per row segment
    constexpr int kStride = kW + 4;       // LDS words per staged segment
    constexpr int kChunks = kW / 4;       // 16-byte chunks per segment
    static_assert(kThreads64 * kStride <= kTiles64 * kTile64, "staging fits the transpose's LDS");
    const int tid = threadIdx.x;          // segment (row tid / 2, tile tid % 2)
    uint4* st = reinterpret_cast<uint4*>(lds + tid * kStride);
#pragma unroll
    for (int k = 0; k < kChunks; ++k) st[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int c = tid + kThreads64 * i;
        const int seg = c / kChunks, k = c % kChunks;
        const int t = seg & 1, row = seg >> 1;
        if ((uint32_t)t < ntile) {
            const uint32_t g = g0 + (uint32_t)t;
            const uint32_t by = fdiv(g, a.bwdiv), bx = g - by * a.bw;
            char* p = a.dst + (int64_t)(by * 64u + (uint32_t)row) * a.dst_pitch + (int64_t)bx * 64 * (int64_t)sizeof(S) +
                      16 * k;
            store16(p, *reinterpret_cast<const uint4*>(lds + seg * kStride + 4 * k));
        }
    }
}

// Factors of column v per log2 d_u - 4 (three classes per column).
__device__ __forceinline__ void column_factors64(const Scale5& t, int v, float (&out)[3]) {
    const int lv = l64(v);
#pragma unroll
    for (int l = 4; l <= 6; ++l) out[l - 4] = pick5(t, l + lv - 8);
}

// Workgroup b of a launch over the plane of `a` (128 threads).  RB bounds
// the zonal size at compile time (r <= RB): the coefficients with u or v >=
// RB are then known zeros, and the inverse passes, unrolled, drop every
// addition of such a zero (a zonal launch takes the least of 8, 16, 32 and
// 64 that holds r).  SAT: the quantiser saturates its levels to int16 (the
// host leaves it out where they provably fit).
template <typename S, int OP, bool STORE, bool SSE, int RB = 64, bool SAT = true>
__device__ __forceinline__ void t64_group(const Args64& a, uint32_t b) {
    __shared__ __align__(16) int32_t lds[kTiles64 * kTile64];
    __shared__ long long red[kThreads64 / 64];
    const int tid = threadIdx.x;
    const uint32_t group = a.spread_rows ? (b % kSpread64) * a.spread_rows + b / kSpread64 : b;
    const uint32_t g0 = group * (uint32_t)kTiles64;
    if (g0 >= a.nblk) return;  // past the last group (interleaved grids only)
    const uint32_t ntile = min((uint32_t)kTiles64, a.nblk - g0);

    // ---- row role: load, forward row pass --------------------------------
    const int rt = tid & 1, rr = tid >> 1;
    const bool rok = (uint32_t)rt < ntile;
    const uint32_t rg = g0 + (uint32_t)(rok ? rt : 0);  // lanes past the plane load a valid tile, unused
    const uint32_t by = fdiv(rg, a.bwdiv), bx = rg - by * a.bw;
    Row64<S> raw;
    load_row64<S>(a.src + (int64_t)(by * 64u + (uint32_t)rr) * a.src_pitch + (int64_t)bx * 64 * (int64_t)sizeof(S),
                  raw);
    {
        int32_t x[64], y[64];
#pragma unroll
        for (int j = 0; j < 64; ++j) x[j] = sample64<S>(raw, j);
        fwd64(x, y);
        int32_t* l = lds + rt * kTile64 + rr * kRow64;
#pragma unroll
        for (int v = 0; v < 64; ++v) l[v] = y[v];
    }
    __syncthreads();

    // ---- column role: forward column pass, coefficient domain -------------
    const int ct = tid >> 6, cv = tid & 63;
    const bool cok = (uint32_t)ct < ntile;
    const uint32_t cg = g0 + (uint32_t)ct;
    int32_t Y[64];
    {
        int32_t c[64];
        const int32_t* l = lds + ct * kTile64 + cv;
#pragma unroll
        for (int i = 0; i < 64; ++i) c[i] = l[i * kRow64];
        fwd64(c, Y);  // Y[u] = coefficient (u, cv)
    }
    if constexpr (STORE && OP != kQuant64) {
        if (cok) {
            int32_t* o = static_cast<int32_t*>(a.cout) + (int64_t)cg * 4096 + cv;
#pragma unroll
            for (int u = 0; u < 64; ++u) o[u * 64] = Y[u];
        }
    }
    if constexpr (OP == kFwd64) return;
    if constexpr (OP == kZonal64) {
        const bool kv = cv < a.r;
        const int lv = l64(cv);
#pragma unroll
        for (int u = 0; u < 64; ++u)
            Y[u] = (u < RB && kv && u < a.r) ? (int32_t)((uint32_t)Y[u] << (12 - l64(u) - lv)) : 0;
    } else {
        float fq[3], fd[3];
        column_factors64(a.qs, cv, fq);
        column_factors64(a.dqs, cv, fd);
        int16_t* o = static_cast<int16_t*>(a.cout) + (int64_t)cg * 4096 + cv;
#pragma unroll
        for (int u = 0; u < 64; ++u) {
            const int32_t q0 = round_away(__fmul_rn((float)Y[u], fq[l64(u) - 4]));
            const int32_t q = SAT ? clamp_i32(q0, -32768, 32767) : q0;
            if constexpr (STORE) {
                if (cok) o[u * 64] = (int16_t)q;
            }
            Y[u] = round_away(__fmul_rn((float)q, fd[l64(u) - 4]));
        }
    }
    if (cv == 0) Y[0] += 2048;  // rounding offset: the DC term reaches every sample with weight 1

    // ---- inverse column pass, transpose, inverse row pass -----------------
    {
        int32_t z[64];
        inv64(Y, z);
        __syncthreads();  // every forward column read of LDS is done
        int32_t* l = lds + ct * kTile64 + cv;
#pragma unroll
        for (int i = 0; i < 64; ++i) l[i * kRow64] = z[i];
    }
    __syncthreads();
    int32_t R[64];
    {
        int32_t c[64];
        const int32_t* l = lds + rt * kTile64 + rr * kRow64;
#pragma unroll
        for (int j = 0; j < 64; ++j) c[j] = j < RB ? l[j] : 0;  // columns v >= RB are zero
        inv64(c, R);
    }
    constexpr int32_t lo = sizeof(S) == 1 ? 0 : -255, hi = 255;
#pragma unroll
    for (int j = 0; j < 64; ++j) R[j] = clamp_i32(R[j] >> 12, lo, hi);
    {
        uint32_t w[Row64<S>::kWords];
        pack_row64<S>(R, w);
        __syncthreads();  // every read of the inverse transpose is done
        store_rows64<S>(lds, w, a, g0, ntile);
    }
    if constexpr (SSE) {
        int32_t s = 0;
        if (rok) {
#pragma unroll
            for (int j = 0; j < 64; ++j) {
                const int32_t e = R[j] - sample64<S>(raw, j);
                s += e * e;
            }
        }
        // one atomic per workgroup when its tiles lie in one image, else
        // one per thread
        const uint32_t last = g0 + ntile - 1u;
        const uint32_t img0 = fdiv(fdiv(g0, a.bwdiv), a.ipbdiv);
        const uint32_t img1 = fdiv(fdiv(last, a.bwdiv), a.ipbdiv);
        if (img0 == img1) {
            const long long v = wave_sum64((long long)s);
            if ((tid & 63) == 0) red[tid >> 6] = v;
            __syncthreads();
            if (tid == 0) {
                const long long t = red[0] + red[1];
                if (t) atomicAdd(a.sse + img0, (unsigned long long)t);
            }
        } else if (rok && s) {
            atomicAdd(a.sse + fdiv(by, a.ipbdiv), (unsigned long long)s);
        }
    }
}

template <typename S, int OP, bool STORE, bool SSE, int RB, bool SAT>
__global__ __launch_bounds__(kThreads64) void k_t64(Args64 a) {
    t64_group<S, OP, STORE, SSE, RB, SAT>(a, blockIdx.x);
}

// T64^T Y T64 per block (block-major int32 in and out).
constexpr int kInvRow64 = 68;                    // output staging: words per row
constexpr int kInvTile64 = 64 * kInvRow64 + 4;   // and per tile

__global__ __launch_bounds__(kThreads64) void k_t64_inv(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                        uint32_t nblk) {
    __shared__ __align__(16) int32_t out_stage[kTiles64 * kInvTile64];
    static_assert(kTiles64 * kTile64 <= kTiles64 * kInvTile64, "the transpose fits the staging array");
    int32_t* lds = out_stage;  // the transpose's [tile][row][65 words] fits the same array
    const int tid = threadIdx.x;
    const uint32_t g0 = blockIdx.x * (uint32_t)kTiles64;
    const uint32_t ntile = min((uint32_t)kTiles64, nblk - g0);
    const int ct = tid >> 6, cv = tid & 63;
    {
        int32_t Y[64], z[64];
        const uint32_t cg = g0 + (uint32_t)((uint32_t)ct < ntile ? ct : 0);
        const int32_t* p = in + (int64_t)cg * 4096 + cv;
#pragma unroll
        for (int u = 0; u < 64; ++u) Y[u] = p[u * 64];
        inv64(Y, z);
        int32_t* l = lds + ct * kTile64 + cv;
#pragma unroll
        for (int i = 0; i < 64; ++i) l[i * kRow64] = z[i];
    }
    __syncthreads();
    const int rt = tid & 1, rr = tid >> 1;
    int32_t c[64], R[64];
    {
        const int32_t* l = lds + rt * kTile64 + rr * kRow64;
#pragma unroll
        for (int j = 0; j < 64; ++j) c[j] = l[j];
    }
    inv64(c, R);
    // the blocks leave through LDS as contiguous 16-byte chunks, whole lines
    // per store instruction ([tile][row][64 words + 4 pad])
    __syncthreads();
    int4* st = reinterpret_cast<int4*>(out_stage + rt * kInvTile64 + rr * kInvRow64);
#pragma unroll
    for (int k = 0; k < 16; ++k) st[k] = make_int4(R[4 * k], R[4 * k + 1], R[4 * k + 2], R[4 * k + 3]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int ch = tid + kThreads64 * i;     // chunk: tile, row, 16-byte piece
        const int t = ch >> 10, row = (ch >> 4) & 63, k = ch & 15;
        if ((uint32_t)t < ntile)
            *reinterpret_cast<int4*>(out + (int64_t)(g0 + (uint32_t)t) * 4096 + row * 64 + 4 * k) =
                *reinterpret_cast<const int4*>(out_stage + t * kInvTile64 + row * kInvRow64 + 4 * k);
    }
}

__global__ __launch_bounds__(256) void k_t64_zero(unsigned long long* p, uint32_t n) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

// Planes of the 64-point calls: sides multiples of 64; 16-byte aligned rows.
int check_plane64(const adct_plane* p) {
    int rc = check_plane(p);
    if (rc) return rc;
    if ((p->height & 63) || (p->width & 63)) return ADCT_E_SHAPE;
    return ADCT_OK;
}

int64_t blocks64(const adct_plane* p) { return (int64_t)(p->height / 64) * (p->width / 64); }

uint32_t grid64(const Args64& a) {
    return a.spread_rows ? a.spread_rows * kSpread64 : (a.nblk + kTiles64 - 1) / kTiles64;
}

template <typename S, int OP, bool STORE, int RB, bool SAT = true>
void launch64_rb(const Args64& a, hipStream_t s) {
    const dim3 grid(grid64(a));
    if (a.sse)
        hipLaunchKernelGGL((k_t64<S, OP, STORE, true, RB, SAT>), grid, dim3(kThreads64), 0, s, a);
    else
        hipLaunchKernelGGL((k_t64<S, OP, STORE, false, RB, SAT>), grid, dim3(kThreads64), 0, s, a);
}

template <typename S, int OP, bool STORE>
void launch64(const Args64& a, hipStream_t s) {
    if constexpr (OP == kZonal64) {
        if (a.r <= 8) return launch64_rb<S, OP, STORE, 8>(a, s);
        if (a.r <= 16) return launch64_rb<S, OP, STORE, 16>(a, s);
        if (a.r <= 32) return launch64_rb<S, OP, STORE, 32>(a, s);
    }
    if constexpr (OP == kQuant64) {
        if (!a.sat) return launch64_rb<S, OP, STORE, 64, false>(a, s);
    }
    launch64_rb<S, OP, STORE, 64>(a, s);
}

template <int OP>
int launch64_typed(int32_t dtype, const Args64& a, hipStream_t s) {
    if (a.nblk == 0) return ADCT_OK;
    if (dtype == ADCT_U8) {
        if (a.cout) launch64<uint8_t, OP, true>(a, s); else launch64<uint8_t, OP, false>(a, s);
    } else {
        if (a.cout) launch64<int16_t, OP, true>(a, s); else launch64<int16_t, OP, false>(a, s);
    }
    return launched();
}

// Shared checks and set-up of the encoders (and the forward call, with no
// destination), then the clear of the SSE output.
int setup64(const adct_plane* src, void* coef, const adct_plane* dst, int32_t image_height, int64_t* sse,
            hipStream_t s, Args64& a) {
    int rc = check_plane64(src);
    if (rc) return rc;
    if (dst) {
        if ((rc = check_plane64(dst))) return rc;
        if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    }
    if (sse && (image_height <= 0 || (image_height & 63) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    if (coef && (((uintptr_t)coef) & 15)) return ADCT_E_ALIGN;
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    if (dst) {
        a.dst = static_cast<char*>(dst->data);
        a.dst_pitch = dst->pitch_bytes;
    }
    a.cout = coef;
    a.nblk = (uint32_t)blocks64(src);
    a.bw = (uint32_t)(src->width / 64);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(sse ? (uint32_t)(image_height / 64) : 1u);
    a.sse = reinterpret_cast<unsigned long long*>(sse);
    if (sse) {
        const uint32_t groups = (a.nblk + kTiles64 - 1) / kTiles64;
        const uint32_t image_tiles = (uint32_t)(image_height / 64) * a.bw;
        if (image_tiles / kTiles64 > kSpreadMin64) a.spread_rows = (groups + kSpread64 - 1) / kSpread64;
        const uint32_t nimg = (uint32_t)(src->height / image_height);
        hipLaunchKernelGGL(k_t64_zero, dim3((nimg + 255) / 256), dim3(256), 0, s, a.sse, nimg);
        return launched();
    }
    return ADCT_OK;
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

int adct_t64_fwd2d(const adct_plane* src, int32_t* coef, void* stream) {
    if (!coef) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args64 a{};
    int rc = setup64(src, coef, nullptr, 0, nullptr, s, a);
    if (rc) return rc;
    return launch64_typed<kFwd64>(src->dtype, a, s);
}

int adct_t64_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream) {
    if (nblk < 0 || nblk > (int64_t)INT32_MAX - kTiles64) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;  // an empty array may be a null pointer
    if (!coef || !out) return ADCT_E_ARG;
    if ((((uintptr_t)coef) & 15) || (((uintptr_t)out) & 15)) return ADCT_E_ALIGN;
    hipLaunchKernelGGL(k_t64_inv, dim3((unsigned)((nblk + kTiles64 - 1) / kTiles64)), dim3(kThreads64), 0,
                       static_cast<hipStream_t>(stream), coef, out, (uint32_t)nblk);
    return launched();
}

int adct_t64_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst, int32_t image_height,
                          int64_t* sse, void* stream) {
    if (r < 0 || r > 64) return ADCT_E_ARG;
    if (!dst) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args64 a{};
    int rc = setup64(src, coef, dst, image_height, sse, s, a);
    if (rc) return rc;
    a.r = r;
    return launch64_typed<kZonal64>(src->dtype, a, s);
}

int adct_t64_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst, int32_t image_height,
                          int64_t* sse, void* stream) {
    float qs[5], dqs[5];
    if (!quant_scales64(qp, qs, dqs)) return ADCT_E_ARG;
    if (!dst) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args64 a{};
    int rc = setup64(src, q, dst, image_height, sse, s, a);
    if (rc) return rc;
    for (int c = 0; c < 5; ++c) {
        a.qs.f[c] = qs[c];
        a.dqs.f[c] = dqs[c];
    }
    a.sat = levels_may_saturate64(src->dtype, qp);
    return launch64_typed<kQuant64>(src->dtype, a, s);
}

}  // extern "C"
