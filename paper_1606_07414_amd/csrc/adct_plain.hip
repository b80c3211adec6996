// Plain and fused device entry points of the C ABI: validate, then launch
// one grid kernel (two when a per-image SSE has to be cleared first) on the
// caller's stream.  Nothing here allocates or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adct_internal.hpp"
#include "adct_core.hpp"
#include "adct_kernels.hpp"
#include "adct_zero.hpp"

namespace adct {
namespace {

Scale5 to_dev(const Scale5Host& h) {
    Scale5 s;
    for (int c = 0; c < 5; ++c) s.f[c] = h.f[c];
    return s;
}

PlaneRef plane_ref(const adct_plane* p) {
    PlaneRef r;
    r.data = static_cast<const char*>(p->data);
    r.pitch = p->pitch_bytes;
    r.bw = (uint32_t)(p->width / 16);
    return r;
}

// Tile-row geometry shared by every plane of a call.
void set_geometry(const adct_plane* p, GroupArgs& a) {
    a.bw = (uint32_t)(p->width / 16);
    a.bwdiv = make_fastdiv(a.bw);
    a.ipbdiv = make_fastdiv(1);
}

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

unsigned elem_grid(uint64_t n4) { return (unsigned)std::min<uint64_t>((n4 + 255) / 256, 1u << 20); }

int check_blocks(const void* p, int64_t nblk) {
    if (nblk < 0 || nblk > (int64_t)INT32_MAX) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;  // an empty array may be a null pointer
    if (!p) return ADCT_E_ARG;
    if (!aligned16(p)) return ADCT_E_ALIGN;
    return ADCT_OK;
}

// Shared argument checks of the reconstruction calls.
int check_recon(const adct_plane* dst, const adct_plane* ref, int32_t image_height, int64_t* sse) {
    int rc = check_plane(dst);
    if (rc) return rc;
    if ((ref == nullptr) != (sse == nullptr)) return ADCT_E_ARG;
    if (ref) {
        if ((rc = check_plane(ref))) return rc;
        if (!same_shape(dst, ref)) return ADCT_E_SHAPE;
        if (image_height <= 0 || (image_height & 15) || dst->height % image_height) return ADCT_E_SHAPE;
        if ((uintptr_t)sse & 7) return ADCT_E_ALIGN;
    }
    return ADCT_OK;
}

// Grid of a plain launch over nblk tiles: groups_per_wg groups per
// workgroup, at least min_gpw; launches that add to the SSE of large images
// interleave their chunks.
struct GroupGrid {
    uint32_t gpw, rows, log2, grid;
};
constexpr uint32_t log2_pow2(uint32_t n) { return n <= 1 ? 0 : 1 + log2_pow2(n >> 1); }

// `shared_lines`: the launch writes uint8 rows whose tile-group segments
// share lines with their neighbours' (kXcdRegions regions, see there).
GroupGrid group_grid(uint32_t nblk, bool sse, uint32_t image_tiles, bool shared_lines = false,
                     uint32_t min_gpw = 1) {
    GroupGrid g;
    g.gpw = groups_per_wg(nblk);
    if (g.gpw < min_gpw) g.gpw = min_gpw;
    const uint32_t span = g.gpw * (uint32_t)kTPW;
    const uint32_t chunks = (nblk + span - 1) / span;
    const uint32_t n = shared_lines ? kXcdRegions : kSseSpread;
    const bool spread = shared_lines || (sse && image_tiles / span > kSseSpreadMin);
    g.log2 = log2_pow2(n);
    g.rows = spread ? (chunks + n - 1) / n : 0u;
    g.grid = g.rows ? g.rows * n : chunks;
    return g;
}

// Host side of shares_lines for a launch's output plane.
template <typename S, typename M>
bool output_shares_lines(const GroupArgs& a) {
    if (M::OUT != kOutSamples || sizeof(S) != 1) return false;
    return (((uintptr_t)a.dst.data | (uint64_t)a.dst.pitch | (uint64_t)a.bw * 16u) & 127u) != 0;
}

template <typename S, typename M>
int launch_group(uint32_t nblk, hipStream_t s, const GroupArgs& a) {
    if (nblk == 0) return ADCT_OK;
    const GroupGrid g = group_grid(nblk, M::SSE && a.sse, a.image_tiles, output_shares_lines<S, M>(a),
                                   prefetch_zone<S, M>()                  ? kZoneGpw
                                   : sse_gathers(M::SSE && a.sse, a.image_tiles) ? kSseGpw
                                                                                 : 1u);
    if (g.gpw == 1)
        hipLaunchKernelGGL((k_group<kTPW, S, M, false>), dim3(g.grid), dim3(kTPW * 8), 0, s, a, nblk, g.gpw, g.rows,
                           g.log2);
    else
        hipLaunchKernelGGL((k_group<kTPW, S, M, true>), dim3(g.grid), dim3(kTPW * 8), 0, s, a, nblk, g.gpw, g.rows,
                           g.log2);
    return launched();
}

template <typename M>
int launch_typed(int32_t dtype, uint32_t nblk, hipStream_t s, const GroupArgs& a) {
    return dtype == ADCT_U8 ? launch_group<uint8_t, M>(nblk, s, a) : launch_group<int16_t, M>(nblk, s, a);
}

// Quantising modes: int16 planes whose levels provably fit skip the
// saturation (kMidQuantFit); uint8 planes never need it, and their kMidQuant
// kernels leave it out.
template <int STORE, int OUT, bool SSE>
int launch_quant(int32_t dtype, bool fit, uint32_t nblk, hipStream_t s, const GroupArgs& a) {
    if (dtype == ADCT_U8) return launch_group<uint8_t, Mode<kInSamples, STORE, kMidQuant, OUT, -1, SSE>>(nblk, s, a);
    if (fit) return launch_group<int16_t, Mode<kInSamples, STORE, kMidQuantFit, OUT, -1, SSE>>(nblk, s, a);
    return launch_group<int16_t, Mode<kInSamples, STORE, kMidQuant, OUT, -1, SSE>>(nblk, s, a);
}

// Zonal modes: uint8 planes get kernels specialised for the common sizes,
// in which the known-zero coefficients fold away.
template <int IN, int STORE, bool SSE>
int launch_zonal(int32_t dtype, int r, uint32_t nblk, hipStream_t s, const GroupArgs& a) {
    if (dtype == ADCT_U8) {
        switch (r) {
            case 2: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, 2, SSE>>(nblk, s, a);
            case 4: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, 4, SSE>>(nblk, s, a);
            case 8: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, 8, SSE>>(nblk, s, a);
            case 12: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, 12, SSE>>(nblk, s, a);
            case 16: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, 16, SSE>>(nblk, s, a);
            default: return launch_group<uint8_t, Mode<IN, STORE, kMidZonal, kOutSamples, -1, SSE>>(nblk, s, a);
        }
    }
    return launch_group<int16_t, Mode<IN, STORE, kMidZonal, kOutSamples, -1, SSE>>(nblk, s, a);
}

// Fills the SSE fields of `a` (no launch).
void sse_fields(const adct_plane* dst, const adct_plane* ref, int32_t image_height, int64_t* sse, GroupArgs& a) {
    a.ipbdiv = make_fastdiv(1);
    if (!sse) return;
    a.ref = plane_ref(ref ? ref : dst);
    a.ipbdiv = make_fastdiv((uint32_t)(image_height / 16));
    a.image_tiles = (uint32_t)(image_height / 16) * (uint32_t)(dst->width / 16);
    a.sse = reinterpret_cast<unsigned long long*>(sse);
}

// Clears the per-image SSE accumulators (a fill kernel, so that the call can
// be captured in a graph) and fills the SSE fields of `a`.
int prepare_sse(const adct_plane* dst, const adct_plane* ref, int32_t image_height, int64_t* sse,
                hipStream_t s, GroupArgs& a) {
    sse_fields(dst, ref, image_height, sse, a);
    if (!sse) return ADCT_OK;
    const uint32_t nimg = (uint32_t)(dst->height / image_height);
    hipLaunchKernelGGL(k_zero_u64, dim3((nimg + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(sse), nimg);
    return launched();
}

template <typename S, typename M>
int launch_planes(const PlaneSet& ps, uint32_t grid, bool pf, hipStream_t s) {
    if (pf)
        hipLaunchKernelGGL((k_group_planes<kTPW, S, M, true>), dim3(grid), dim3(kTPW * 8), 0, s, ps);
    else
        hipLaunchKernelGGL((k_group_planes<kTPW, S, M, false>), dim3(grid), dim3(kTPW * 8), 0, s, ps);
    return launched();
}

template <int STORE, bool SSE>
int launch_quant_planes(int32_t dtype, bool fit, const PlaneSet& ps, uint32_t grid, bool pf, hipStream_t s) {
    if (dtype == ADCT_U8)
        return launch_planes<uint8_t, Mode<kInSamples, STORE, kMidQuant, kOutSamples, -1, SSE>>(ps, grid, pf, s);
    if (fit)
        return launch_planes<int16_t, Mode<kInSamples, STORE, kMidQuantFit, kOutSamples, -1, SSE>>(ps, grid, pf, s);
    return launch_planes<int16_t, Mode<kInSamples, STORE, kMidQuant, kOutSamples, -1, SSE>>(ps, grid, pf, s);
}

}  // namespace
}  // namespace adct

using namespace adct;

extern "C" {

int adct_fwd2d(const adct_plane* src, int32_t* coef, void* stream) {
    int rc = check_plane(src);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(src);
    if ((rc = check_blocks(coef, nblk))) return rc;
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.cout = coef;
    return launch_typed<Mode<kInSamples, kStoreY, kMidNone, kOutNothing, -1, false>>(
        src->dtype, (uint32_t)nblk, static_cast<hipStream_t>(stream), a);
}

int adct_fwd2d_quant(const adct_plane* src, int qp, int16_t* q, void* stream) {
    int rc = check_plane(src);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(src);
    if ((rc = check_blocks(q, nblk))) return rc;
    Scale5Host qs;
    if (!quant_scales(qp, &qs, nullptr)) return ADCT_E_ARG;
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.cout = q;
    a.qs = to_dev(qs);
    return launch_quant<kStoreQ, kOutNothing, false>(src->dtype, i16_levels_fit(qs), (uint32_t)nblk,
                                                     static_cast<hipStream_t>(stream), a);
}

int adct_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(out, nblk))) return rc;
    GroupArgs a{};
    a.cin = coef;
    a.bout = out;
    a.bw = 1;
    a.bwdiv = make_fastdiv(1);
    a.ipbdiv = make_fastdiv(1);
    return launch_group<int16_t, Mode<kInZfix, kStoreNone, kMidNone, kOutBlocks, -1, false>>(
        (uint32_t)nblk, static_cast<hipStream_t>(stream), a);
}

int adct_scale(const int32_t* coef, int64_t nblk, float* out, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(out, nblk))) return rc;
    if (nblk == 0) return ADCT_OK;
    Scale5Host ss;
    ortho_scales(&ss);
    const uint64_t n4 = (uint64_t)nblk * 64;
    hipLaunchKernelGGL(k_scale, dim3(elem_grid(n4)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const int4*>(coef), reinterpret_cast<float4*>(out), n4, to_dev(ss));
    return launched();
}

int adct_quant(const int32_t* coef, int64_t nblk, int qp, int16_t* q, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(q, nblk))) return rc;
    Scale5Host qs;
    if (!quant_scales(qp, &qs, nullptr)) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;
    const uint64_t n4 = (uint64_t)nblk * 64;
    hipLaunchKernelGGL(k_quant, dim3(elem_grid(n4)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const int4*>(coef), reinterpret_cast<short4*>(q), n4, to_dev(qs));
    return launched();
}

int adct_dequant(const int16_t* q, int64_t nblk, int qp, int32_t* zfix, void* stream) {
    int rc;
    if ((rc = check_blocks(q, nblk)) || (rc = check_blocks(zfix, nblk))) return rc;
    Scale5Host dqs;
    if (!quant_scales(qp, nullptr, &dqs)) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;
    const uint64_t n4 = (uint64_t)nblk * 64;
    hipLaunchKernelGGL(k_dequant, dim3(elem_grid(n4)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const short4*>(q), reinterpret_cast<int4*>(zfix), n4, to_dev(dqs));
    return launched();
}

int adct_zonal(const int32_t* coef, int64_t nblk, int r, int32_t* zfix, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(zfix, nblk))) return rc;
    if (r < 0 || r > 16) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;
    const uint64_t n4 = (uint64_t)nblk * 64;
    hipLaunchKernelGGL(k_zonal, dim3(elem_grid(n4)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const int4*>(coef), reinterpret_cast<int4*>(zfix), n4, r);
    return launched();
}

int adct_zigzag(const int32_t* coef, int64_t nblk, int r, int32_t* zfix, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(zfix, nblk))) return rc;
    if (r < 0 || r > 256) return ADCT_E_ARG;
    if (nblk == 0) return ADCT_OK;
    const uint64_t n4 = (uint64_t)nblk * 64;
    hipLaunchKernelGGL(k_zigzag, dim3(elem_grid(n4)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const int4*>(coef), reinterpret_cast<int4*>(zfix), n4, r);
    return launched();
}

int adct_recon(const int32_t* zfix, const adct_plane* dst, void* stream) {
    int rc = check_plane(dst);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(dst);
    if ((rc = check_blocks(zfix, nblk))) return rc;
    GroupArgs a{};
    a.cin = zfix;
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    return launch_typed<Mode<kInZfix, kStoreNone, kMidNone, kOutSamples, -1, false>>(
        dst->dtype, (uint32_t)nblk, static_cast<hipStream_t>(stream), a);
}

int adct_zonal_recon(const int32_t* coef, int r, const adct_plane* dst, const adct_plane* ref,
                     int32_t image_height, int64_t* sse, void* stream) {
    if (r < 0 || r > 16) return ADCT_E_ARG;
    int rc = check_recon(dst, ref, image_height, sse);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(dst);
    if ((rc = check_blocks(coef, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.cin = coef;
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.r = r;
    if ((rc = prepare_sse(dst, ref, image_height, sse, s, a))) return rc;
    return sse ? launch_zonal<kInY, kStoreNone, true>(dst->dtype, r, (uint32_t)nblk, s, a)
               : launch_zonal<kInY, kStoreNone, false>(dst->dtype, r, (uint32_t)nblk, s, a);
}

int adct_zigzag_recon(const int32_t* coef, int r, const adct_plane* dst, const adct_plane* ref,
                      int32_t image_height, int64_t* sse, void* stream) {
    if (r < 0 || r > 256) return ADCT_E_ARG;
    int rc = check_recon(dst, ref, image_height, sse);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(dst);
    if ((rc = check_blocks(coef, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.cin = coef;
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.r = r;
    if ((rc = prepare_sse(dst, ref, image_height, sse, s, a))) return rc;
    return sse ? launch_typed<Mode<kInY, kStoreNone, kMidZigzag, kOutSamples, -1, true>>(dst->dtype, (uint32_t)nblk, s, a)
               : launch_typed<Mode<kInY, kStoreNone, kMidZigzag, kOutSamples, -1, false>>(dst->dtype, (uint32_t)nblk, s, a);
}

int adct_dequant_recon(const int16_t* q, int qp, const adct_plane* dst, const adct_plane* ref,
                       int32_t image_height, int64_t* sse, void* stream) {
    Scale5Host dqs;
    if (!quant_scales(qp, nullptr, &dqs)) return ADCT_E_ARG;
    int rc = check_recon(dst, ref, image_height, sse);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(dst);
    if ((rc = check_blocks(q, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.cin = q;
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.dqs = to_dev(dqs);
    if ((rc = prepare_sse(dst, ref, image_height, sse, s, a))) return rc;
    return sse ? launch_typed<Mode<kInQ, kStoreNone, kMidDequant, kOutSamples, -1, true>>(dst->dtype, (uint32_t)nblk, s, a)
               : launch_typed<Mode<kInQ, kStoreNone, kMidDequant, kOutSamples, -1, false>>(dst->dtype, (uint32_t)nblk, s, a);
}

int adct_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                      int32_t image_height, int64_t* sse, void* stream) {
    if (r < 0 || r > 16) return ADCT_E_ARG;
    int rc = check_plane(src);
    if (rc) return rc;
    if ((rc = check_plane(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (sse && (image_height <= 0 || (image_height & 15) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    const int64_t nblk = plane_blocks(src);
    if (coef && (rc = check_blocks(coef, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.cout = coef;
    a.r = r;
    if ((rc = prepare_sse(dst, src, image_height, sse, s, a))) return rc;
    const uint32_t n = (uint32_t)nblk;
    if (coef)
        return sse ? launch_zonal<kInSamples, kStoreY, true>(src->dtype, r, n, s, a)
                   : launch_zonal<kInSamples, kStoreY, false>(src->dtype, r, n, s, a);
    return sse ? launch_zonal<kInSamples, kStoreNone, true>(src->dtype, r, n, s, a)
               : launch_zonal<kInSamples, kStoreNone, false>(src->dtype, r, n, s, a);
}

int adct_encode_zigzag(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                       int32_t image_height, int64_t* sse, void* stream) {
    if (r < 0 || r > 256) return ADCT_E_ARG;
    int rc = check_plane(src);
    if (rc) return rc;
    if ((rc = check_plane(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (sse && (image_height <= 0 || (image_height & 15) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    const int64_t nblk = plane_blocks(src);
    if (coef && (rc = check_blocks(coef, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.cout = coef;
    a.r = r;
    if ((rc = prepare_sse(dst, src, image_height, sse, s, a))) return rc;
    const uint32_t n = (uint32_t)nblk;
    const int32_t dt = src->dtype;
    if (coef)
        return sse ? launch_typed<Mode<kInSamples, kStoreY, kMidZigzag, kOutSamples, -1, true>>(dt, n, s, a)
                   : launch_typed<Mode<kInSamples, kStoreY, kMidZigzag, kOutSamples, -1, false>>(dt, n, s, a);
    return sse ? launch_typed<Mode<kInSamples, kStoreNone, kMidZigzag, kOutSamples, -1, true>>(dt, n, s, a)
               : launch_typed<Mode<kInSamples, kStoreNone, kMidZigzag, kOutSamples, -1, false>>(dt, n, s, a);
}

int adct_compare_encode(const adct_plane* src, int32_t transform, int32_t retention, int r, const adct_plane* dst,
                        int32_t image_height, int64_t* sse, void* stream) {
    if (retention != ADCT_KEEP_ZONAL && retention != ADCT_KEEP_ZIGZAG) return ADCT_E_ARG;
    if (r < 0 || r > (retention == ADCT_KEEP_ZONAL ? 16 : 256)) return ADCT_E_ARG;
    if (transform != ADCT_XF_PROPOSED && transform != ADCT_XF_WHT && transform != ADCT_XF_DCT) return ADCT_E_ARG;
    int rc = check_plane(src);
    if (rc) return rc;
    if ((rc = check_plane(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (sse && (image_height <= 0 || (image_height & 15) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    if (transform == ADCT_XF_PROPOSED)
        return retention == ADCT_KEEP_ZONAL ? adct_encode_zonal(src, r, nullptr, dst, image_height, sse, stream)
                                            : adct_encode_zigzag(src, r, nullptr, dst, image_height, sse, stream);
    if (transform == ADCT_XF_DCT) return launch_dct_codec(src, retention, r, dst, image_height, sse, stream);
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.r = r;
    if ((rc = prepare_sse(dst, src, image_height, sse, s, a))) return rc;
    const uint32_t n = (uint32_t)plane_blocks(src);
    const int32_t dt = src->dtype;
    if (retention == ADCT_KEEP_ZONAL)
        return sse ? launch_typed<Mode<kInSamples, kStoreNone, kMidZonal, kOutSamples, -1, true, kXfWht>>(dt, n, s, a)
                   : launch_typed<Mode<kInSamples, kStoreNone, kMidZonal, kOutSamples, -1, false, kXfWht>>(dt, n, s, a);
    return sse ? launch_typed<Mode<kInSamples, kStoreNone, kMidZigzag, kOutSamples, -1, true, kXfWht>>(dt, n, s, a)
               : launch_typed<Mode<kInSamples, kStoreNone, kMidZigzag, kOutSamples, -1, false, kXfWht>>(dt, n, s, a);
}

int adct_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst, int32_t image_height,
                      int64_t* sse, void* stream) {
    Scale5Host qs, dqs;
    if (!quant_scales(qp, &qs, &dqs)) return ADCT_E_ARG;
    int rc = check_plane(src);
    if (rc) return rc;
    if ((rc = check_plane(dst))) return rc;
    if (!same_shape(src, dst)) return ADCT_E_SHAPE;
    if (sse && (image_height <= 0 || (image_height & 15) || src->height % image_height)) return ADCT_E_SHAPE;
    if (sse && ((uintptr_t)sse & 7)) return ADCT_E_ALIGN;
    const int64_t nblk = plane_blocks(src);
    if (q && (rc = check_blocks(q, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GroupArgs a{};
    a.src = plane_ref(src);
    set_geometry(src, a);
    a.dst = plane_ref(dst);
    set_geometry(dst, a);
    a.cout = q;
    a.qs = to_dev(qs);
    a.dqs = to_dev(dqs);
    if ((rc = prepare_sse(dst, src, image_height, sse, s, a))) return rc;
    const uint32_t n = (uint32_t)nblk;
    const int32_t dt = src->dtype;
    const bool fit = i16_levels_fit(qs);
    if (q)
        return sse ? launch_quant<kStoreQ, kOutSamples, true>(dt, fit, n, s, a)
                   : launch_quant<kStoreQ, kOutSamples, false>(dt, fit, n, s, a);
    return sse ? launch_quant<kStoreNone, kOutSamples, true>(dt, fit, n, s, a)
               : launch_quant<kStoreNone, kOutSamples, false>(dt, fit, n, s, a);
}

int adct_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, int32_t block, void* stream) {
    if (!jobs || njobs < 1 || njobs > ADCT_MAX_PLANES) return ADCT_E_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (block == 8) return t8_encode_quant_planes(jobs, njobs, qp, stream);
    if (block == 32) return t32_encode_quant_planes(jobs, njobs, qp, stream);
    if (block != 16) return ADCT_E_ARG;
    Scale5Host qs, dqs;
    if (!quant_scales(qp, &qs, &dqs)) return ADCT_E_ARG;
    static_assert(ADCT_MAX_PLANES <= kMaxPlanes, "one launch holds every plane");
    const bool store = jobs[0].q != nullptr, want_sse = jobs[0].sse != nullptr;
    const int32_t dt = jobs[0].src.dtype;
    PlaneSet ps{};
    ZeroSet<ADCT_MAX_PLANES> zs{};
    uint64_t grid = 0;
    bool pf = false;
    for (int32_t i = 0; i < njobs; ++i) {
        const adct_quant_job& j = jobs[i];
        int rc = check_plane(&j.src);
        if (rc) return rc;
        if ((rc = check_plane(&j.dst))) return rc;
        if (!same_shape(&j.src, &j.dst)) return ADCT_E_SHAPE;
        if (j.src.dtype != dt || (j.q != nullptr) != store || (j.sse != nullptr) != want_sse) return ADCT_E_ARG;
        if (want_sse) {
            if (j.image_height <= 0 || (j.image_height & 15) || j.src.height % j.image_height) return ADCT_E_SHAPE;
            if ((uintptr_t)j.sse & 7) return ADCT_E_ALIGN;
        }
        const int64_t nblk = plane_blocks(&j.src);
        if (store && (rc = check_blocks(j.q, nblk))) return rc;
        PlaneLaunch& pl = ps.p[i];
        GroupArgs& a = pl.a;
        a.src = plane_ref(&j.src);
        set_geometry(&j.src, a);
        a.dst = plane_ref(&j.dst);
        a.cout = j.q;
        a.qs = to_dev(qs);
        a.dqs = to_dev(dqs);
        sse_fields(&j.dst, &j.src, j.image_height, j.sse, a);
        const bool shared =
            dt == ADCT_U8 && (((uintptr_t)a.dst.data | (uint64_t)a.dst.pitch | (uint64_t)a.bw * 16u) & 127u) != 0;
        const GroupGrid g = group_grid((uint32_t)nblk, want_sse, a.image_tiles, shared,
                                       sse_gathers(want_sse, a.image_tiles) ? kSseGpw : 1u);
        pl.nblk = (uint32_t)nblk;
        pl.gpw = g.gpw;
        pl.spread_rows = g.rows;
        pl.spread_log2 = g.log2;
        pl.first_wg = (uint32_t)grid;
        grid += g.grid;
        pf = pf || g.gpw > 1;
        if (want_sse) {
            zs.p[i] = reinterpret_cast<unsigned long long*>(j.sse);
            zs.n[i] = (uint32_t)(j.src.height / j.image_height);
        }
    }
    if (grid > (uint64_t)INT32_MAX) return ADCT_E_TOO_LARGE;
    ps.n = (uint32_t)njobs;
    if (want_sse) {
        zs.count = (uint32_t)njobs;
        clear_sets(zs, s);
        if (int rc = launched()) return rc;
    }
    const bool fit = i16_levels_fit(qs);
    if (store)
        return want_sse ? launch_quant_planes<kStoreQ, true>(dt, fit, ps, (uint32_t)grid, pf, s)
                        : launch_quant_planes<kStoreQ, false>(dt, fit, ps, (uint32_t)grid, pf, s);
    return want_sse ? launch_quant_planes<kStoreNone, true>(dt, fit, ps, (uint32_t)grid, pf, s)
                    : launch_quant_planes<kStoreNone, false>(dt, fit, ps, (uint32_t)grid, pf, s);
}

int adct_sse(const adct_plane* a, const adct_plane* b, int32_t image_height, int64_t* sse, void* stream) {
    int rc;
    if ((rc = check_plane(a)) || (rc = check_plane(b))) return rc;
    if (!same_shape(a, b)) return ADCT_E_SHAPE;
    if (!sse) return ADCT_E_ARG;
    if ((uintptr_t)sse & 7) return ADCT_E_ALIGN;
    if (image_height <= 0 || (image_height & 15) || a->height % image_height) return ADCT_E_SHAPE;
    const uint64_t segs_per_row = (uint64_t)(a->width / 16);
    const uint64_t nseg = (uint64_t)a->height * segs_per_row;
    if (nseg >= (1ull << 32) - 256) return ADCT_E_SHAPE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t nimg = (uint32_t)(a->height / image_height);
    hipLaunchKernelGGL(k_zero_u64, dim3((nimg + 255) / 256), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(sse), nimg);
    const unsigned grid = (unsigned)((nseg + 255) / 256);
    if (a->dtype == ADCT_U8)
        hipLaunchKernelGGL(k_sse<uint8_t>, dim3(grid), dim3(256), 0, s, plane_ref(a), plane_ref(b),
                           (uint32_t)nseg, (uint32_t)segs_per_row, (uint32_t)image_height,
                           reinterpret_cast<unsigned long long*>(sse));
    else
        hipLaunchKernelGGL(k_sse<int16_t>, dim3(grid), dim3(256), 0, s, plane_ref(a), plane_ref(b),
                           (uint32_t)nseg, (uint32_t)segs_per_row, (uint32_t)image_height,
                           reinterpret_cast<unsigned long long*>(sse));
    return launched();
}

}  // extern "C"
