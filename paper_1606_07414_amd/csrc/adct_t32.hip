// The 32x32 codec of the 32-point extension T32 (butterflies in
// adct_t32_common.hpp): forward transform, zonal retention or quantisation
// with S folded in, inverse, rounding and the per-image SSE, one pass.
//
// A workgroup of 256 threads codes 8 consecutive tiles (raster order).
//   row role     rt = tid % 8, rr = tid / 8: row rr of tile rt, so the 8
//                lanes of one sample row read 8 horizontally adjacent
//                32-sample segments (contiguous for tiles of one tile row)
//   column role  ct = tid / 32, cv = tid % 32: column cv of tile ct, so the
//                32 lanes of a half-wave touch 32 adjacent coefficients of
//                one row of a block (one contiguous 128-byte run for int32)
// The row pass runs in registers and goes to LDS ([tile][row][33 words],
// tile stride 1060 words: both roles' accesses are free of bank
// conflicts); the column pass, the coefficient domain and the inverse
// column pass run in the column role; the inverse row pass in the row role
// again after a second LDS transpose.  Coefficients and levels are stored
// straight from the column role: for each frequency u, a half-wave writes
// one contiguous row of a block.
//
// Fixed point: the weights 1024 / (d_u d_v) make T32^T (W . T32 X T32^T) T32
// = 1024 X exact; reconstructions are rounded as floor((R + 512) / 1024).
#include <hip/hip_runtime.h>

#include "adct_core.hpp"
#include "adct_internal.hpp"
#include "adct_round.hpp"
#include "adct_t32_common.hpp"
#include "adct_tile.hpp"
#include "adct_zero.hpp"

namespace adct {
namespace {

enum Op32 { kFwd32 = 0, kZonal32 = 1, kQuant32 = 2 };

struct Args32 {
    const char* src;
    int64_t src_pitch;
    char* dst;
    int64_t dst_pitch;
    void* cout;              // int32 Y (forward, zonal) or int16 levels (quant); null: not stored
    uint32_t nblk, bw;       // tiles, tiles per tile row
    FastDiv bwdiv, ipbdiv;   // / bw, / tile rows per image
    int32_t r;               // zonal size
    Scale5 qs, dqs;          // per class c = log2 d_u + log2 d_v - 6
    unsigned long long* sse; // per image, or null
    uint32_t spread_rows;    // 0: workgroup b takes group b; else interleaved (see k_t32)
    bool sat;                // quantising: levels may leave int16 and are saturated (host side)
};

// Whether the levels of a 32x32 quantising call can leave int16.  A level is
// at most sqrt(d_u d_v) |x|max / Delta <= 32 |x|max / Delta (entries of T32
// in {0, +1, -1}, d_u of them nonzero in row u): for uint8 samples 8160 /
// Delta, within int16 at every QP; for int16 samples within +-2047 it is
// 65504 / Delta, within int16 from QP 10 (Delta = 2) on.
bool levels_may_saturate32(int32_t dtype, int qp) { return dtype != ADCT_U8 && qp < 10; }

constexpr int kTiles32 = 8;                // tiles per workgroup
constexpr int kRow32 = 33;                 // LDS words per staged row
constexpr int kTile32 = 32 * kRow32 + 4;   // LDS words per staged tile
// Workgroups of a launch that adds to the SSE of large images are dealt
// over the plane in this many interleaved streams (as the 16-point group
// kernel does), so that the workgroups resident at one time add to several
// images' sums instead of queueing on the atomics of one, while each stream
// stays a sequential sweep of its part of the plane.
constexpr uint32_t kSpread32 = 4;
constexpr uint32_t kSpreadMin32 = 64;      // groups of 8 tiles per image

// Raw words of one 32-sample row (uint8: 8 words, int16: 16) and their
// samples as int32.
template <typename S>
struct Row32 {
    static constexpr int kWords = 8 * (int)sizeof(S);
    uint32_t w[kWords];
};

template <typename S>
__device__ __forceinline__ void load_row32(const char* p, Row32<S>& r) {
#pragma unroll
    for (int k = 0; k < Row32<S>::kWords / 4; ++k) {
        const uint4 v = reinterpret_cast<const uint4*>(p)[k];
        r.w[4 * k] = v.x;
        r.w[4 * k + 1] = v.y;
        r.w[4 * k + 2] = v.z;
        r.w[4 * k + 3] = v.w;
    }
}

template <typename S>
__device__ __forceinline__ int32_t sample32(const Row32<S>& r, int j) {
    if constexpr (sizeof(S) == 1)
        return (int32_t)((r.w[j >> 2] >> (8 * (j & 3))) & 0xffu);
    else
        return (j & 1) ? ((int32_t)r.w[j >> 1] >> 16) : (int32_t)(int16_t)(r.w[j >> 1] & 0xffffu);
}

// The 32 output samples of a row as raw words, the layout of Row32.
template <typename S>
__device__ __forceinline__ void pack_row32(const int32_t (&o)[32], uint32_t (&w)[Row32<S>::kWords]) {
    if constexpr (sizeof(S) == 1) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            w[i] = (uint32_t)o[4 * i] | ((uint32_t)o[4 * i + 1] << 8) | ((uint32_t)o[4 * i + 2] << 16) |
                   ((uint32_t)o[4 * i + 3] << 24);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) w[i] = ((uint32_t)o[2 * i] & 0xffffu) | ((uint32_t)o[2 * i + 1] << 16);
    }
}

// Output rows leave through LDS: each thread stages its packed row, then the
// workgroup stores 16-byte chunks with consecutive threads on consecutive
// chunks of a sample row (all 8 tiles' segments of that row in turn), so
// every store instruction writes whole contiguous lines.  Stored straight
// from the row role, each lane's row would go out as 2 (uint8) or 4 (int16)
// pieces at a 32- or 64-byte stride, half or a quarter of each line per
// instruction, which non-temporal stores do not merge: measured on MI355X,
// the int16 codec ran 3 to 4.5 times slower that way.
template <typename S>
__device__ __forceinline__ void store_rows32(int32_t* lds, const uint32_t (&w)[Row32<S>::kWords], const Args32& a,
                                             uint32_t g0, uint32_t ntile) {
    constexpr int kW = Row32<S>::kWords;  // words per row segment
    constexpr int kStride = kW + 4;       // LDS words per staged segment
    constexpr int kChunks = kW / 4;       // 16-byte chunks per segment
    const int tid = threadIdx.x;          // segment (row tid / 8, tile tid % 8)
    uint4* st = reinterpret_cast<uint4*>(lds + tid * kStride);
#pragma unroll
    for (int k = 0; k < kChunks; ++k) st[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kChunks; ++i) {
        const int c = tid + 256 * i;
        const int seg = c / kChunks, k = c % kChunks;
        const int t = seg & 7, row = seg >> 3;
        if ((uint32_t)t < ntile) {
            const uint32_t g = g0 + (uint32_t)t;
            const uint32_t by = fdiv(g, a.bwdiv), bx = g - by * a.bw;
            char* p = a.dst + (int64_t)(by * 32u + (uint32_t)row) * a.dst_pitch + (int64_t)bx * 32 * (int64_t)sizeof(S) +
                      16 * k;
            store16(p, *reinterpret_cast<const uint4*>(lds + seg * kStride + 4 * k));
        }
    }
}

// Factors of column v per log2 d_u - 3 (three classes per column).
__device__ __forceinline__ void column_factors32(const Scale5& t, int v, float (&out)[3]) {
    const int lv = l32(v);
#pragma unroll
    for (int l = 3; l <= 5; ++l) out[l - 3] = pick5(t, l + lv - 6);
}

// Workgroup b of a launch over the plane of `a` (256 threads).  RB bounds
// the zonal size at compile time (r <= RB): the coefficients with u or v >=
// RB are then known zeros, and the inverse passes, unrolled, drop every
// addition of such a zero (a zonal launch without a coefficient output
// takes the least of 8, 16 and 32 that holds r).  SAT: the quantiser
// saturates its levels to int16 (the host leaves it out where they provably
// fit).
template <typename S, int OP, bool STORE, bool SSE, int RB = 32, bool SAT = true>
__device__ __forceinline__ void t32_group(const Args32& a, uint32_t b) {
    __shared__ __align__(16) int32_t lds[kTiles32 * kTile32];
    __shared__ long long red[4];
    const int tid = threadIdx.x;
    const uint32_t group = a.spread_rows ? (b % kSpread32) * a.spread_rows + b / kSpread32 : b;
    const uint32_t g0 = group * (uint32_t)kTiles32;
    if (g0 >= a.nblk) return;  // past the last group (interleaved grids only)
    const uint32_t ntile = min((uint32_t)kTiles32, a.nblk - g0);

    // ---- row role: load, forward row pass --------------------------------
    const int rt = tid & 7, rr = tid >> 3;
    const bool rok = (uint32_t)rt < ntile;
    const uint32_t rg = g0 + (uint32_t)(rok ? rt : 0);  // lanes past the plane load a valid tile, unused
    const uint32_t by = fdiv(rg, a.bwdiv), bx = rg - by * a.bw;
    Row32<S> raw;
    load_row32<S>(a.src + (int64_t)(by * 32u + (uint32_t)rr) * a.src_pitch + (int64_t)bx * 32 * (int64_t)sizeof(S),
                  raw);
    {
        int32_t x[32], y[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) x[j] = sample32<S>(raw, j);
        fwd32(x, y);
        int32_t* l = lds + rt * kTile32 + rr * kRow32;
#pragma unroll
        for (int v = 0; v < 32; ++v) l[v] = y[v];
    }
    __syncthreads();

    // ---- column role: forward column pass, coefficient domain -------------
    const int ct = tid >> 5, cv = tid & 31;
    const bool cok = (uint32_t)ct < ntile;
    const uint32_t cg = g0 + (uint32_t)ct;
    int32_t Y[32];
    {
        int32_t c[32];
        const int32_t* l = lds + ct * kTile32 + cv;
#pragma unroll
        for (int i = 0; i < 32; ++i) c[i] = l[i * kRow32];
        fwd32(c, Y);  // Y[u] = coefficient (u, cv)
    }
    if constexpr (STORE && OP != kQuant32) {
        if (cok) {
            int32_t* o = static_cast<int32_t*>(a.cout) + (int64_t)cg * 1024 + cv;
#pragma unroll
            for (int u = 0; u < 32; ++u) o[u * 32] = Y[u];
        }
    }
    if constexpr (OP == kFwd32) return;
    if constexpr (OP == kZonal32) {
        const bool kv = cv < a.r;
        const int lv = l32(cv);
#pragma unroll
        for (int u = 0; u < 32; ++u)
            Y[u] = (u < RB && kv && u < a.r) ? (int32_t)((uint32_t)Y[u] << (10 - l32(u) - lv)) : 0;
    } else {
        float fq[3], fd[3];
        column_factors32(a.qs, cv, fq);
        column_factors32(a.dqs, cv, fd);
        int16_t* o = static_cast<int16_t*>(a.cout) + (int64_t)cg * 1024 + cv;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            const int32_t q0 = round_away(__fmul_rn((float)Y[u], fq[l32(u) - 3]));
            const int32_t q = SAT ? clamp_i32(q0, -32768, 32767) : q0;
            if constexpr (STORE) {
                if (cok) o[u * 32] = (int16_t)q;
            }
            Y[u] = round_away(__fmul_rn((float)q, fd[l32(u) - 3]));
        }
    }
    if (cv == 0) Y[0] += 512;  // rounding offset: the DC term reaches every sample with weight 1

    // ---- inverse column pass, transpose, inverse row pass -----------------
    {
        int32_t z[32];
        inv32(Y, z);
        __syncthreads();  // every forward column read of LDS is done
        int32_t* l = lds + ct * kTile32 + cv;
#pragma unroll
        for (int i = 0; i < 32; ++i) l[i * kRow32] = z[i];
    }
    __syncthreads();
    int32_t R[32];
    {
        int32_t c[32];
        const int32_t* l = lds + rt * kTile32 + rr * kRow32;
#pragma unroll
        for (int j = 0; j < 32; ++j) c[j] = j < RB ? l[j] : 0;  // columns v >= RB are zero
        inv32(c, R);
    }
    constexpr int32_t lo = sizeof(S) == 1 ? 0 : -255, hi = 255;
#pragma unroll
    for (int j = 0; j < 32; ++j) R[j] = clamp_i32(R[j] >> 10, lo, hi);
    {
        uint32_t w[Row32<S>::kWords];
        pack_row32<S>(R, w);
        __syncthreads();  // every read of the inverse transpose is done
        store_rows32<S>(lds, w, a, g0, ntile);
    }
    if constexpr (SSE) {
        int32_t s = 0;
        if (rok) {
#pragma unroll
            for (int j = 0; j < 32; ++j) {
                const int32_t e = R[j] - sample32<S>(raw, j);
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
                const long long t = red[0] + red[1] + red[2] + red[3];
                if (t) atomicAdd(a.sse + img0, (unsigned long long)t);
            }
        } else if (rok && s) {
            atomicAdd(a.sse + fdiv(by, a.ipbdiv), (unsigned long long)s);
        }
    }
}

// T32^T Y T32 per block (block-major int32 in and out).
constexpr int kInvRow = 36;                     // output staging: words per row
constexpr int kInvTile = 32 * kInvRow + 4;      // and per tile

template <typename S, int OP, bool STORE, bool SSE, int RB, bool SAT>
__global__ __launch_bounds__(256) void k_t32(Args32 a) {
    t32_group<S, OP, STORE, SSE, RB, SAT>(a, blockIdx.x);
}

// Several planes in one launch: plane i takes the workgroups from first[i]
// (ascending) up to the next plane's, as k_t32 would over that plane alone.
struct Set32 {
    Args32 p[ADCT_MAX_PLANES];
    uint32_t first[ADCT_MAX_PLANES];
    uint32_t n;
};

template <typename S, int OP, bool STORE, bool SSE, bool SAT>
__global__ __launch_bounds__(256) void k_t32_planes(Set32 ps) {
    uint32_t i = 0;
#pragma unroll
    for (uint32_t k = 1; k < (uint32_t)ADCT_MAX_PLANES; ++k)
        if (k < ps.n && blockIdx.x >= ps.first[k]) i = k;
    t32_group<S, OP, STORE, SSE, 32, SAT>(ps.p[i], blockIdx.x - ps.first[i]);
}

__global__ __launch_bounds__(256) void k_t32_inv(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                uint32_t nblk) {
    __shared__ __align__(16) int32_t out_stage[kTiles32 * kInvTile];
    int32_t* lds = out_stage;  // the transpose's [tile][row][33 words] fits the same array
    const int tid = threadIdx.x;
    const uint32_t g0 = blockIdx.x * (uint32_t)kTiles32;
    const uint32_t ntile = min((uint32_t)kTiles32, nblk - g0);
    const int ct = tid >> 5, cv = tid & 31;
    {
        int32_t Y[32], z[32];
        const uint32_t cg = g0 + (uint32_t)((uint32_t)ct < ntile ? ct : 0);
        const int32_t* p = in + (int64_t)cg * 1024 + cv;
#pragma unroll
        for (int u = 0; u < 32; ++u) Y[u] = p[u * 32];
        inv32(Y, z);
        int32_t* l = lds + ct * kTile32 + cv;
#pragma unroll
        for (int i = 0; i < 32; ++i) l[i * kRow32] = z[i];
    }
    __syncthreads();
    const int rt = tid & 7, rr = tid >> 3;
    int32_t c[32], R[32];
    {
        const int32_t* l = lds + rt * kTile32 + rr * kRow32;
#pragma unroll
        for (int j = 0; j < 32; ++j) c[j] = l[j];
    }
    inv32(c, R);
    // the blocks leave through LDS as contiguous 16-byte chunks, whole lines
    // per store instruction ([tile][row][32 words + 4 pad], tile stride
    // 1156 words)
    __syncthreads();
    int4* st = reinterpret_cast<int4*>(out_stage + rt * kInvTile + rr * kInvRow);
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] = make_int4(R[4 * k], R[4 * k + 1], R[4 * k + 2], R[4 * k + 3]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int ch = tid + 256 * i;
        const int t = ch >> 8, row = (ch >> 3) & 31, k = ch & 7;
        if ((uint32_t)t < ntile)
            *reinterpret_cast<int4*>(out + (int64_t)(g0 + (uint32_t)t) * 1024 + row * 32 + 4 * k) =
                *reinterpret_cast<const int4*>(out_stage + t * kInvTile + row * kInvRow + 4 * k);
    }
}

__global__ __launch_bounds__(256) void k_t32_zero(unsigned long long* p, uint32_t n) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t < n) p[t] = 0ull;
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

// Planes of the 32-point calls: sides multiples of 32; 16-byte aligned rows.
int check_plane32(const adct_plane* p) {
    int rc = check_plane(p);
    if (rc) return rc;
    if ((p->height & 31) || (p->width & 31)) return ADCT_E_SHAPE;
    return ADCT_OK;
}

int64_t blocks32(const adct_plane* p) { return (int64_t)(p->height / 32) * (p->width / 32); }

uint32_t grid32(const Args32& a) {
    return a.spread_rows ? a.spread_rows * kSpread32 : (a.nblk + kTiles32 - 1) / kTiles32;
}

template <typename S, int OP, bool STORE, int RB, bool SAT = true>
void launch32_rb(const Args32& a, hipStream_t s) {
    const dim3 grid(grid32(a));
    if (a.sse)
        hipLaunchKernelGGL((k_t32<S, OP, STORE, true, RB, SAT>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_t32<S, OP, STORE, false, RB, SAT>), grid, dim3(256), 0, s, a);
}

template <typename S, int OP, bool STORE>
void launch32(const Args32& a, hipStream_t s) {
    // The bound pays where the launch is bound by issue, without the
    // coefficient output (r = 8: 196 against 160 us on 1024 images of 512^2).
    // With it the launch streams 6 KB per block, and the bounded kernels were
    // the slower ones: 300-302 against 280-285 us at r = 4 and 8.
    if constexpr (OP == kZonal32 && !STORE) {
        if (a.r <= 8) return launch32_rb<S, OP, STORE, 8>(a, s);
        if (a.r <= 16) return launch32_rb<S, OP, STORE, 16>(a, s);
    }
    if constexpr (OP == kQuant32) {
        if (!a.sat) return launch32_rb<S, OP, STORE, 32, false>(a, s);
    }
    launch32_rb<S, OP, STORE, 32>(a, s);
}

template <int OP>
int launch32_typed(int32_t dtype, const Args32& a, hipStream_t s) {
    if (a.nblk == 0) return ADCT_OK;
    if (dtype == ADCT_U8) {
        if (a.cout) launch32<uint8_t, OP, true>(a, s); else launch32<uint8_t, OP, false>(a, s);
    } else {
        if (a.cout) launch32<int16_t, OP, true>(a, s); else launch32<int16_t, OP, false>(a, s);
    }
    return launched();
}

// Shared checks and argument set-up of the encoders (and the forward call,
// with no destination); no launch.
int setup_args32(const adct_plane* src, void* coef, const adct_plane* dst, int32_t image_height, int64_t* sse,
                 Args32& a) {
    int rc = check_plane32(src);
    if (rc) return rc;
    if (dst) {
        if ((rc = check_plane32(dst))) return rc;
        if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    }
    if (sse && (image_height <= 0 || (image_height & 31) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    if (coef && (((uintptr_t)coef) & 15)) return ADCT_E_ALIGN;
    a.src = static_cast<const char*>(src->data);
    a.src_pitch = src->pitch_bytes;
    if (dst) {
        a.dst = static_cast<char*>(dst->data);
        a.dst_pitch = dst->pitch_bytes;
    }
    a.cout = coef;
    a.nblk = (uint32_t)blocks32(src);
    a.bw = (uint32_t)(src->width / 32);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(sse ? (uint32_t)(image_height / 32) : 1u);
    a.sse = reinterpret_cast<unsigned long long*>(sse);
    if (sse) {
        const uint32_t groups = (a.nblk + kTiles32 - 1) / kTiles32;
        const uint32_t image_tiles = (uint32_t)(image_height / 32) * a.bw;
        if (image_tiles / kTiles32 > kSpreadMin32) a.spread_rows = (groups + kSpread32 - 1) / kSpread32;
    }
    return ADCT_OK;
}

// The same, then the clear of the SSE output.
int setup32(const adct_plane* src, void* coef, const adct_plane* dst, int32_t image_height, int64_t* sse,
            hipStream_t s, Args32& a) {
    const int rc = setup_args32(src, coef, dst, image_height, sse, a);
    if (rc || !sse) return rc;
    const uint32_t nimg = (uint32_t)(src->height / image_height);
    hipLaunchKernelGGL(k_t32_zero, dim3((nimg + 255) / 256), dim3(256), 0, s, a.sse, nimg);
    return launched();
}

template <typename S, bool STORE, bool SSE>
void launch32_planes(const Set32& ps, uint32_t grid, hipStream_t s) {
    // every plane of the set has the same sample type and QP
    if (ps.p[0].sat)
        hipLaunchKernelGGL((k_t32_planes<S, kQuant32, STORE, SSE, true>), dim3(grid), dim3(256), 0, s, ps);
    else
        hipLaunchKernelGGL((k_t32_planes<S, kQuant32, STORE, SSE, false>), dim3(grid), dim3(256), 0, s, ps);
}

template <typename S>
void launch32_planes_typed(const Set32& ps, uint32_t grid, bool store, bool sse, hipStream_t s) {
    if (store) {
        if (sse) launch32_planes<S, true, true>(ps, grid, s); else launch32_planes<S, true, false>(ps, grid, s);
    } else {
        if (sse) launch32_planes<S, false, true>(ps, grid, s); else launch32_planes<S, false, false>(ps, grid, s);
    }
}

}  // namespace

int t32_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, void* stream) {
    float qs[5], dqs[5];
    if (!quant_scales32(qp, qs, dqs)) return ADCT_E_ARG;
    const bool store = jobs[0].q != nullptr, want_sse = jobs[0].sse != nullptr;
    const int32_t dt = jobs[0].src.dtype;
    Set32 ps{};
    ZeroSet<ADCT_MAX_PLANES> zs{};
    uint64_t grid = 0;
    for (int32_t i = 0; i < njobs; ++i) {
        const adct_quant_job& j = jobs[i];
        if (j.src.dtype != dt || (j.q != nullptr) != store || (j.sse != nullptr) != want_sse) return ADCT_E_ARG;
        Args32& a = ps.p[i];
        const int rc = setup_args32(&j.src, j.q, &j.dst, j.image_height, j.sse, a);
        if (rc) return rc;
        for (int c = 0; c < 5; ++c) {
            a.qs.f[c] = qs[c];
            a.dqs.f[c] = dqs[c];
        }
        a.sat = levels_may_saturate32(dt, qp);
        ps.first[i] = (uint32_t)grid;
        grid += grid32(a);
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
        launch32_planes_typed<uint8_t>(ps, (uint32_t)grid, store, want_sse, s);
    else
        launch32_planes_typed<int16_t>(ps, (uint32_t)grid, store, want_sse, s);
    return launched();
}

}  // namespace adct

using namespace adct;

extern "C" {

int adct_t32_fwd2d(const adct_plane* src, int32_t* coef, void* stream) {
    if (!coef) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args32 a{};
    int rc = setup32(src, coef, nullptr, 0, nullptr, s, a);
    if (rc) return rc;
    return launch32_typed<kFwd32>(src->dtype, a, s);
}

int adct_t32_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream) {
    if (nblk < 0 || nblk > (int64_t)INT32_MAX - kTiles32) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;  // an empty array may be a null pointer
    if (!coef || !out) return ADCT_E_ARG;
    if ((((uintptr_t)coef) & 15) || (((uintptr_t)out) & 15)) return ADCT_E_ALIGN;
    hipLaunchKernelGGL(k_t32_inv, dim3((unsigned)((nblk + kTiles32 - 1) / kTiles32)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), coef, out, (uint32_t)nblk);
    return launched();
}

int adct_t32_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst, int32_t image_height,
                          int64_t* sse, void* stream) {
    if (r < 0 || r > 32) return ADCT_E_ARG;
    if (!dst) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args32 a{};
    int rc = setup32(src, coef, dst, image_height, sse, s, a);
    if (rc) return rc;
    a.r = r;
    return launch32_typed<kZonal32>(src->dtype, a, s);
}

int adct_t32_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst, int32_t image_height,
                          int64_t* sse, void* stream) {
    float qs[5], dqs[5];
    if (!quant_scales32(qp, qs, dqs)) return ADCT_E_ARG;
    if (!dst) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Args32 a{};
    int rc = setup32(src, q, dst, image_height, sse, s, a);
    if (rc) return rc;
    for (int c = 0; c < 5; ++c) {
        a.qs.f[c] = qs[c];
        a.dqs.f[c] = dqs[c];
    }
    a.sat = levels_may_saturate32(src->dtype, qp);
    return launch32_typed<kQuant32>(src->dtype, a, s);
}

}  // extern "C"
