// Internal declarations shared by the library's translation units.
#pragma once

#include <stdint.h>

#include "adct.h"
#include "adct_butterfly.hpp"

namespace adct {

// Host mirror of the device Scale5 (five per-class factors).
struct Scale5Host {
    float f[5];
};

// Quantiser / dequantiser factors per class for `qp` (false if out of range).
bool quant_scales(int qp, Scale5Host* qs, Scale5Host* dqs);
// Whether every quantisation level of an int16 plane (samples within
// [-2047, 2047]) fits int16 with the 16-point quantiser factors `qs`, so that
// the saturation to int16 can be left out (true from QP 4 on).
bool i16_levels_fit(const Scale5Host& qs);
// fp32(s_u s_v) per class.
void ortho_scales(Scale5Host* ss);
// class c = log2 d_u + log2 d_v - 4 of coefficient (u, v).
int class_of(int u, int v);

// Exact-DCT comparison codec (adct_compare.hip); arguments already checked.
int launch_dct_codec(const adct_plane* src, int32_t kind, int r, const adct_plane* dst, int32_t image_height,
                     int64_t* sse, void* stream);

// adct_encode_quant_planes for 8x8 blocks with T8 (adct_t8.hip) and 32x32
// blocks with T32 (adct_t32.hip); njobs already checked against
// ADCT_MAX_PLANES.
int t8_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, void* stream);
int t32_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, void* stream);

inline int sample_bytes(int32_t dtype) { return dtype == ADCT_U8 ? 1 : dtype == ADCT_I16 ? 2 : 0; }

// Validate a plane descriptor (see the conventions in adct.h).
inline int check_plane(const adct_plane* p) {
    if (!p || !p->data) return ADCT_E_ARG;
    const int sz = sample_bytes(p->dtype);
    if (!sz) return ADCT_E_DTYPE;
    if (p->height <= 0 || p->width <= 0 || (p->height & 15) || (p->width & 15)) return ADCT_E_SHAPE;
    if (p->pitch_bytes < (int64_t)p->width * sz) return ADCT_E_SHAPE;
    if ((p->pitch_bytes & 15) || (((uintptr_t)p->data) & 15)) return ADCT_E_ALIGN;
    const int64_t nblk = (int64_t)(p->height / 16) * (p->width / 16);
    if (nblk > (int64_t)INT32_MAX) return ADCT_E_SHAPE;
    return ADCT_OK;
}

inline int64_t plane_blocks(const adct_plane* p) { return (int64_t)(p->height / 16) * (p->width / 16); }

inline bool same_shape(const adct_plane* a, const adct_plane* b) {
    return a->dtype == b->dtype && a->height == b->height && a->width == b->width;
}

inline bool aligned16(const void* p) { return (((uintptr_t)p) & 15) == 0; }

}  // namespace adct
