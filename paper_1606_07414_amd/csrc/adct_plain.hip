// Plain and fused device entry points of the C ABI: validate, then launch
// one grid kernel (two when a per-image SSE has to be cleared first) on the
// caller's stream.  Nothing here allocates or synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adct_internal.hpp"
#include "adct_kernels.hpp"

namespace adct {
namespace {

constexpr int kTPW = 16;  // tiles per workgroup of the plain grid kernels

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

int launched() { return hipGetLastError() == hipSuccess ? ADCT_OK : ADCT_E_HIP; }

unsigned tile_grid(int64_t nblk) { return (unsigned)((nblk + kTPW - 1) / kTPW); }

unsigned elem_grid(uint64_t n4) { return (unsigned)std::min<uint64_t>((n4 + 255) / 256, 1u << 20); }

int check_blocks(const void* p, int64_t nblk) {
    if (!p || nblk < 0 || nblk > (int64_t)INT32_MAX) return ADCT_E_ARG;
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

template <int IN, int OUT, bool SSE>
void launch_inv_typed(int32_t dtype, unsigned grid, hipStream_t s, const InvArgs& a) {
    if (dtype == ADCT_U8)
        hipLaunchKernelGGL((k_inv<kTPW, uint8_t, IN, OUT, SSE>), dim3(grid), dim3(kTPW * 16), 0, s, a);
    else
        hipLaunchKernelGGL((k_inv<kTPW, int16_t, IN, OUT, SSE>), dim3(grid), dim3(kTPW * 16), 0, s, a);
}

template <int IN>
int recon_common(const void* in, const Scale5Host* dqs, int r, const adct_plane* dst, const adct_plane* ref,
                 int32_t image_height, int64_t* sse, void* stream) {
    int rc = check_recon(dst, ref, image_height, sse);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(dst);
    if ((rc = check_blocks(in, nblk))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    InvArgs a{};
    a.in = in;
    a.nblk = (uint32_t)nblk;
    a.r = r;
    if (dqs) a.dqs = to_dev(*dqs);
    a.dst = plane_ref(dst);
    const unsigned grid = tile_grid(nblk);
    if (sse) {
        const uint32_t nimg = (uint32_t)(dst->height / image_height);
        hipLaunchKernelGGL(k_zero_u64, dim3((nimg + 255) / 256), dim3(256), 0, s,
                           reinterpret_cast<unsigned long long*>(sse), nimg);
        a.ref = plane_ref(ref);
        a.ipb = (uint32_t)(image_height / 16);
        a.sse = reinterpret_cast<unsigned long long*>(sse);
        launch_inv_typed<IN, kOutPlane, true>(dst->dtype, grid, s, a);
    } else {
        a.ipb = 1;
        launch_inv_typed<IN, kOutPlane, false>(dst->dtype, grid, s, a);
    }
    return launched();
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
    FwdArgs a{};
    a.src = plane_ref(src);
    a.nblk = (uint32_t)nblk;
    a.out = coef;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (src->dtype == ADCT_U8)
        hipLaunchKernelGGL((k_fwd<kTPW, uint8_t, kOutCoef>), dim3(tile_grid(nblk)), dim3(kTPW * 16), 0, s, a);
    else
        hipLaunchKernelGGL((k_fwd<kTPW, int16_t, kOutCoef>), dim3(tile_grid(nblk)), dim3(kTPW * 16), 0, s, a);
    return launched();
}

int adct_fwd2d_quant(const adct_plane* src, int qp, int16_t* q, void* stream) {
    int rc = check_plane(src);
    if (rc) return rc;
    const int64_t nblk = plane_blocks(src);
    if ((rc = check_blocks(q, nblk))) return rc;
    Scale5Host qs;
    if (!quant_scales(qp, &qs, nullptr)) return ADCT_E_ARG;
    FwdArgs a{};
    a.src = plane_ref(src);
    a.nblk = (uint32_t)nblk;
    a.out = q;
    a.qs = to_dev(qs);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (src->dtype == ADCT_U8)
        hipLaunchKernelGGL((k_fwd<kTPW, uint8_t, kOutQuant>), dim3(tile_grid(nblk)), dim3(kTPW * 16), 0, s, a);
    else
        hipLaunchKernelGGL((k_fwd<kTPW, int16_t, kOutQuant>), dim3(tile_grid(nblk)), dim3(kTPW * 16), 0, s, a);
    return launched();
}

int adct_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream) {
    int rc;
    if ((rc = check_blocks(coef, nblk)) || (rc = check_blocks(out, nblk))) return rc;
    if (nblk == 0) return ADCT_OK;
    InvArgs a{};
    a.in = coef;
    a.nblk = (uint32_t)nblk;
    a.out_block = out;
    a.ipb = 1;
    hipLaunchKernelGGL((k_inv<kTPW, int16_t, kInZfix, kOutBlock, false>), dim3(tile_grid(nblk)),
                       dim3(kTPW * 16), 0, static_cast<hipStream_t>(stream), a);
    return launched();
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

int adct_recon(const int32_t* zfix, const adct_plane* dst, void* stream) {
    return recon_common<kInZfix>(zfix, nullptr, 16, dst, nullptr, 0, nullptr, stream);
}

int adct_zonal_recon(const int32_t* coef, int r, const adct_plane* dst, const adct_plane* ref,
                     int32_t image_height, int64_t* sse, void* stream) {
    if (r < 0 || r > 16) return ADCT_E_ARG;
    return recon_common<kInZonal>(coef, nullptr, r, dst, ref, image_height, sse, stream);
}

int adct_dequant_recon(const int16_t* q, int qp, const adct_plane* dst, const adct_plane* ref,
                       int32_t image_height, int64_t* sse, void* stream) {
    Scale5Host dqs;
    if (!quant_scales(qp, nullptr, &dqs)) return ADCT_E_ARG;
    return recon_common<kInDequant>(q, &dqs, 16, dst, ref, image_height, sse, stream);
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
