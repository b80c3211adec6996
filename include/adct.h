/*
 * adct.h -- C ABI of the MI355X (gfx950) blockwise 16-point multiplierless
 * approximate DCT library (libadct.so).
 *
 * The method: Silveira et al., "Multiplierless 16-point DCT approximation
 * for low-complexity image and video coding".  A 16x16 matrix T over
 * {0, +1, -1} (Section 2.1) is applied to every disjoint 16x16 block A of a
 * plane as Y = T A T^T (Section 3.1), each 1D pass with the 44-addition
 * factorisation T = P2 M4 M3 M2 P1 M1 (Section 2.2).  The orthogonalising
 * diagonal S = sqrt((T T^T)^-1) (Section 2.1) is never applied as a separate
 * step: it is folded into the quantisation / dequantisation scale factors
 * or into the zonal weights (Section 2.1, last paragraph).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: ADCT_OK (0) or a negative ADCT_E_* code; adct_strerror()
 *   names it.  Arguments are validated before anything is launched; a call
 *   that returns an error has launched nothing.
 * - "Device" pointers are HIP device (or managed) memory owned by the
 *   caller.  Plain calls never allocate, never synchronise, and are
 *   asynchronous on `stream` (a hipStream_t passed as void*; NULL = the
 *   legacy default stream).  Faults inside a kernel surface at the caller's
 *   next synchronisation of that stream.
 * - Plain calls keep no state and may be issued from several host threads.
 * - Planes (adct_plane) are row-major with a byte pitch; height and width
 *   are positive multiples of 16 (else ADCT_E_SHAPE); the pitch is at least
 *   width * sample size and a multiple of the sample size.  Sample (0,0)
 *   must be 16-byte aligned and the pitch a multiple of 16 bytes.
 * - Coefficient-domain arrays are block-major: [nblk][16][16], block
 *   k = by * (width/16) + bx in raster order, element u*16 + v, u the
 *   vertical and v the horizontal frequency.  They must be 16-byte aligned.
 *   A call on nblk == 0 blocks launches nothing and returns ADCT_OK once its
 *   other arguments are valid; its array pointers may then be NULL.
 * - A batch of equally sized images is passed as one tall plane (images
 *   stacked vertically); `image_height` then names each image's height so
 *   that per-image sums of squared errors can be formed.
 */
#ifndef ADCT_H
#define ADCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADCT_ABI_VERSION 2

/* ---- status codes ---------------------------------------------------- */
#define ADCT_OK            0
#define ADCT_PENDING       1   /* adct_server_poll: request not finished yet  */
#define ADCT_E_ARG        -1   /* null / out-of-range argument                */
#define ADCT_E_SHAPE      -2   /* side not a positive multiple of 16, pitch   */
#define ADCT_E_DTYPE      -3   /* sample type not supported by this call      */
#define ADCT_E_HIP        -4   /* a HIP runtime call failed                   */
#define ADCT_E_NOMEM      -5   /* library-owned allocation failed             */
#define ADCT_E_TOO_LARGE  -6   /* request can never fit the server's pool     */
#define ADCT_E_STOPPED    -7   /* server stopped; request cancelled           */
#define ADCT_E_TIMEOUT    -8   /* bounded wait expired                        */
#define ADCT_E_NOTFOUND   -9   /* unknown ticket / tuning entry               */
#define ADCT_E_ALIGN     -10   /* pointer or pitch misaligned                 */

/* ---- sample types ---------------------------------------------------- */
#define ADCT_U8   1   /* uint8 image samples, reconstruction clamped to [0,255]    */
#define ADCT_I16  2   /* int16 residual samples, reconstruction clamped to [-255,255] */

typedef struct adct_plane {
    void*   data;        /* device pointer to sample (0,0)                 */
    int32_t dtype;       /* ADCT_U8 or ADCT_I16                            */
    int32_t height;      /* rows, positive multiple of 16                  */
    int32_t width;       /* samples per row, positive multiple of 16       */
    int32_t reserved;
    int64_t pitch_bytes; /* bytes from one row to the next                 */
} adct_plane;

/* ---- host-side information ---------------------------------------------- */

/* Message for a status code (static string, never NULL). */
const char* adct_strerror(int code);

/* ADCT_ABI_VERSION of the loaded library. */
int adct_abi_version(void);

/* Waits for the work queued on `stream` and reports whether it, or an
 * earlier HIP call of this host thread, failed: ADCT_OK, or ADCT_E_HIP (the
 * thread's HIP error state is then cleared).  The one call besides the
 * batch, server and autotuner calls that synchronises. */
int adct_check(void* stream);

/* Host copies of the library's constants (Section 2.1): T (row-major,
 * T[u*16+j]), the diagonal s of S = sqrt((T T^T)^-1), and the zonal weights
 * W[u*16+v] = 256 / (d_u d_v), d = diag(T T^T).  Any pointer may be NULL. */
int adct_constants(int32_t* T256, double* s16, int32_t* W256);

/* Host run of the kernels' fp32 rounding (round half away from zero, the
 * rule of the quantiser and dequantiser) against (int32_t)roundf for the
 * fp32 values with bit patterns first_bits .. first_bits + count - 1
 * (NaNs, infinities and values outside int32 skipped): *mismatches
 * receives the number that differ.  A check, not a compute call. */
int adct_round_check(uint32_t first_bits, uint32_t count, int64_t* mismatches);

/* Host copy of the zig-zag ranks the kernels use (Section 3.1's retention
 * order): rank256[u*16+v] = position of coefficient (u, v) in the scan
 * (see adct_zigzag).  ADCT_E_ARG for NULL. */
int adct_zigzag_ranks(int32_t* rank256);

/* Host copies of the quantisation tables for `qp` (Section 2.1: S merged
 * into the quantiser).  Step Delta = 2^((qp-4)/6), qp in [0, 63].
 *   qs[u*16+v]  = fp32(s_u s_v / Delta)        (forward scale)
 *   dqs[u*16+v] = fp32(256 Delta s_u s_v)      (dequantise to 8 fractional bits)
 * Both are computed in double and rounded once to float.  Either pointer may
 * be NULL.  ADCT_E_ARG for qp outside [0, 63]. */
int adct_quant_tables(int qp, float* qs256, float* dqs256);

/* PSNR per image from exact sums of squared errors (host arrays):
 * out[i] = 10 log10(peak^2 * pixels_per_image / sse[i]), +inf when sse is 0. */
int adct_psnr(const int64_t* sse, int32_t n, double pixels_per_image, double peak,
              double* out);

/* The kernels' own 1D butterflies executed on the host (the same source the
 * GPU runs): X = T x (which = 0) or x = T^T X (which = 1), Section 2.2's
 * 44-addition dataflow, the comparison WHT X = H x (which = 2, natural
 * order, 64 additions), or the 8-point T8 (which = 3) or T8^T (which = 4)
 * applied to each half of the 16 values (14 additions each), as the 8x8 and
 * mixed codecs apply it.  For checking the dataflows without a GPU.
 * in16, out16: host int32[16]; ADCT_E_ARG for another `which`. */
int adct_host_butterfly(int32_t which, const int32_t* in16, int32_t* out16);

/* The same butterflies as adct_host_butterfly (same `which`), run on the
 * host with a value type that counts every addition and subtraction it
 * takes part in and defines no other arithmetic: *additions receives the
 * count for the whole call (Table 1: 44 for T and for T^T by the Section 2.2
 * factorisation, 64 for the WHT; the T8 modes transform both halves, 2 x 14).
 * ADCT_E_ARG for a NULL pointer, another `which`, or a result outside int32. */
int adct_host_butterfly_count(int32_t which, const int32_t* in16, int32_t* out16, int64_t* additions);

/* ---- plain device calls -------------------------------------------------- */

/* Forward transform Y = T A T^T of every 16x16 block of `src` (Section 3.1;
 * each 1D pass by the Section 2.2 factorisation, 44 additions).
 * src: U8 or I16 plane.  coef: device int32 [nblk][16][16].
 * Exact (bit-identical to the integer matrix product) for every U8 input
 * (|Y| <= 65280) and for I16 samples within [-2047, 2047] (the row pass runs
 * in 16-bit lanes); I16 samples outside that range give unspecified
 * coefficients.  The same range rule holds for every call taking an I16
 * source plane. */
int adct_fwd2d(const adct_plane* src, int32_t* coef, void* stream);

/* Plain inverse R = T^T Y T of `nblk` blocks (Section 3.1, without S).
 * coef, out: device int32 [nblk][16][16].  Exact while every |R| < 2^31
 * (guaranteed for |Y| < 2^25); otherwise wraps modulo 2^32.  Because
 * T^T T is not diagonal this is not the inverse of adct_fwd2d; see
 * adct_zonal / adct_dequant for the S-weighted inverse path. */
int adct_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream);

/* Orthonormal coefficients B = S Y S (Section 2.1, C-hat = S T):
 * out[k][u][v] = fp32(Y) * fp32(s_u s_v), one rounding each.
 * coef: device int32, out: device float32, both [nblk][16][16]. */
int adct_scale(const int32_t* coef, int64_t nblk, float* out, void* stream);

/* Quantisation levels with S folded in (Section 2.1; uniform step
 * Delta = 2^((qp-4)/6), round half away from zero, no dead zone):
 * q = round(fp32(Y) * qs[u][v]) saturated to int16.  coef: device int32,
 * q: device int16, [nblk][16][16]. */
int adct_quant(const int32_t* coef, int64_t nblk, int qp, int16_t* q, void* stream);

/* Dequantisation to 8 fractional bits with S folded in:
 * zfix = round(fp32(q) * dqs[u][v]) (half away from zero), int32.
 * q: device int16, zfix: device int32, [nblk][16][16]. */
int adct_dequant(const int16_t* q, int64_t nblk, int qp, int32_t* zfix, void* stream);

/* Zonal retention of the top-left r x r coefficients (Section 3.1), S folded
 * in as zfix = Y * W[u][v] for u < r and v < r, 0 elsewhere
 * (W = 256/(d_u d_v), a left shift by 0..4).  r in [0, 16].
 * coef, zfix: device int32 [nblk][16][16]. */
int adct_zonal(const int32_t* coef, int64_t nblk, int r, int32_t* zfix, void* stream);

/* Zig-zag retention of the first r coefficients of each block (Section 3.1:
 * the experiment keeps the first r elements of the zig-zag sequence, r up to
 * 150), S folded in as for adct_zonal: zfix = Y * W[u][v] where the rank of
 * (u, v) in the scan is below r, 0 elsewhere.  The scan is the JPEG zig-zag
 * extended to 16x16 (anti-diagonals u + v in turn, u rising on odd and
 * falling on even ones).  r in [0, 256].  coef, zfix: device int32
 * [nblk][16][16]. */
int adct_zigzag(const int32_t* coef, int64_t nblk, int r, int32_t* zfix, void* stream);

/* Reconstruction from 8-fractional-bit coefficients (Section 3.1 inverse):
 * R = T^T zfix T per block, sample = clamp(floor((R + 128) / 256)) to
 * [0, 255] (U8) or [-255, 255] (I16), written into the plane `dst`, whose
 * shape fixes nblk.  zfix: device int32 [nblk][16][16]; exact while
 * |R| < 2^31. */
int adct_recon(const int32_t* zfix, const adct_plane* dst, void* stream);

/* Exact per-image sums of squared differences between two planes of the same
 * shape and type; images are the consecutive bands of `image_height` rows
 * (a positive multiple of 16 dividing the plane height).
 * sse: device int64 [height / image_height], overwritten. */
int adct_sse(const adct_plane* a, const adct_plane* b, int32_t image_height,
             int64_t* sse, void* stream);

/* ---- fused device calls (one pass over HBM each) --------------------- */

/* adct_fwd2d followed by adct_quant, without storing Y. */
int adct_fwd2d_quant(const adct_plane* src, int qp, int16_t* q, void* stream);

/* adct_zonal followed by adct_recon, and -- when `ref` and `sse` are both
 * non-NULL -- adct_sse of the reconstruction against `ref` (same shape and
 * type as dst) with images of `image_height` rows.  Only the kept r x r
 * coefficients of each block are read.  dst may alias nothing else. */
int adct_zonal_recon(const int32_t* coef, int r, const adct_plane* dst,
                     const adct_plane* ref, int32_t image_height, int64_t* sse,
                     void* stream);

/* adct_zigzag followed by adct_recon (and the optional SSE, as above).  Only
 * the block rows and columns that hold kept coefficients are read. */
int adct_zigzag_recon(const int32_t* coef, int r, const adct_plane* dst,
                      const adct_plane* ref, int32_t image_height, int64_t* sse,
                      void* stream);

/* adct_dequant followed by adct_recon (and the optional SSE, as above). */
int adct_dequant_recon(const int16_t* q, int qp, const adct_plane* dst,
                       const adct_plane* ref, int32_t image_height, int64_t* sse,
                       void* stream);

/* Single-pass encoder with reconstruction, zonal form (Section 3.1's
 * experiment): per block Y = T A T^T, optionally stored to `coef` (as
 * adct_fwd2d; NULL skips the store), then zonal retention of the top-left
 * r x r coefficients with S folded in, the inverse, rounding and clamping
 * into `dst` (same shape and type as src), and -- when `sse` is non-NULL --
 * the exact per-image SSE of dst against src for images of `image_height`
 * rows.  Bit-identical to adct_fwd2d + adct_zonal_recon; reads src once.
 * r in [0, 16].  sse: device int64 [height / image_height], overwritten. */
int adct_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                      int32_t image_height, int64_t* sse, void* stream);

/* Single-pass encoder with reconstruction, zig-zag form (Section 3.1's
 * experiment as the paper runs it): as adct_encode_zonal with the first r
 * coefficients of the zig-zag scan kept (adct_zigzag).  Bit-identical to
 * adct_fwd2d + adct_zigzag_recon.  r in [0, 256]. */
int adct_encode_zigzag(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                       int32_t image_height, int64_t* sse, void* stream);

/* Single-pass encoder with reconstruction, quantised form (Section 3.2's
 * use, S folded into the quantiser): levels q as adct_fwd2d_quant, stored to
 * `q` unless NULL, then dequantisation, inverse, rounding and clamping into
 * `dst`, and the optional per-image SSE against src.  Bit-identical to
 * adct_fwd2d_quant + adct_dequant_recon. */
int adct_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst,
                      int32_t image_height, int64_t* sse, void* stream);

/* Quantising single-pass encoders over several planes at one QP in one
 * launch (with one clear of every SSE output before it): the planes of a
 * video frame stack (Y, U and V, which differ in size), or any other set.
 * block selects the transform and block size:
 *   16  T on 16x16 blocks, each job coded exactly as adct_encode_quant;
 *    8  T8 on 8x8 blocks, as adct_t8_encode_quant;
 *   32  T32 on 32x32 blocks, as adct_t32_encode_quant;
 * with that call's plane rules, level layout ([blocks][block][block], block
 * rows in raster order) and image heights (multiples of block).  Results are
 * bit-identical to the per-plane call; the short launches of small planes
 * no longer each fill and drain the device on their own.  All jobs must have
 * the same dtype, and either all or none of them store levels (q) and SSE.
 * njobs in [1, ADCT_MAX_PLANES].  Jobs must not overlap in their outputs. */
#define ADCT_MAX_PLANES 8

typedef struct adct_quant_job {
    adct_plane src;          /* samples in                                      */
    adct_plane dst;          /* reconstruction out, same shape and type as src  */
    int16_t* q;              /* levels out, block-major, or NULL                */
    int64_t* sse;            /* per-image SSE [src.height / image_height], or NULL */
    int32_t image_height;    /* rows per image when sse is set                  */
    int32_t reserved;
} adct_quant_job;

int adct_encode_quant_planes(const adct_quant_job* jobs, int32_t njobs, int qp, int32_t block, void* stream);

/* ---- comparison transforms through the same codec ----------------------- */
/* Tables 1 and 2 compare the approximation with the exact DCT and with the
 * Walsh-Hadamard transform; this call runs any of the three through Section
 * 3.1's codec on 16x16 blocks: forward, retention, inverse, rounding half up
 * and clamping into dst, and the optional exact per-image SSE.
 *   ADCT_XF_PROPOSED  T, as adct_encode_zonal / adct_encode_zigzag (bit-exact).
 *   ADCT_XF_WHT       natural-order Hadamard H (H[k][j] = (-1)^popcount(k&j)),
 *                     integer and exact: H H^T = 16 I, so the normalisation
 *                     weights are all 1 and R = H^T Z H carries 8 fractional
 *                     bits; 64 additions per 16-point pass.
 *   ADCT_XF_DCT       the orthonormal DCT-II C in fp32 on the matrix cores:
 *                     B = C A C^T, retention, X = C^T B C, output
 *                     clamp(floor(X + 1/2)).  Differs from a float64
 *                     evaluation only where X lies within about 1e-3 of a
 *                     rounding boundary.
 * retention: ADCT_KEEP_ZONAL (top-left r x r, r in [0, 16]) or
 * ADCT_KEEP_ZIGZAG (first r of the zig-zag scan, r in [0, 256]).  Planes as
 * for adct_encode_zonal (U8 or I16); no coefficients are written. */
#define ADCT_XF_PROPOSED 0
#define ADCT_XF_WHT      1
#define ADCT_XF_DCT      2
#define ADCT_KEEP_ZONAL  0
#define ADCT_KEEP_ZIGZAG 1

int adct_compare_encode(const adct_plane* src, int32_t transform, int32_t retention, int r, const adct_plane* dst,
                        int32_t image_height, int64_t* sse, void* stream);

/* ---- the 8-point transform T8 on 8x8 blocks ---------------------------- */
/* T is built from two instances of the 8-point approximation T8 (Section
 * 2.1); the instance on the sum path of the factorisation (Section 2.2) is
 * T8[k][j] = T[2k][j], j < 8 (the even rows of T act on x_j + x_{15-j}
 * only), computed with 14 additions.  Section 3.2's second scenario codes
 * with both the 8- and the 16-point transform; these calls are the 8-point
 * codec on disjoint 8x8 blocks, with S8 = diag(T8 T8^T)^(-1/2) folded in as
 * for the 16-point calls: zonal weights W8 = 64 / (d_u d_v), quantiser
 * tables qs = fp32(s_u s_v / Delta) and dqs = fp32(64 Delta s_u s_v), and
 * reconstruction clamp(floor((R + 32) / 64)).  Planes: sides multiples of 8
 * (else ADCT_E_SHAPE); sample (0,0) and the pitch aligned to 8 bytes for
 * U8 and 16 bytes for I16 (else ADCT_E_ALIGN); coefficient arrays
 * are block-major [nblk8][8][8] with block k = by * (width/8) + bx,
 * element u*8 + v, 16-byte aligned.  image_height: a multiple of 8. */

/* Host copies of T8 (row-major), the diagonal of S8 and W8. */
int adct_t8_constants(int32_t* T64, double* s8, int32_t* W64);

/* Host copies of the 8-point quantisation tables for `qp` in [0, 63]. */
int adct_t8_quant_tables(int qp, float* qs64, float* dqs64);

/* Y = T8 A T8^T for every 8x8 block A of src (U8 or I16); coef: device
 * int32 [nblk8][8][8]. */
int adct_t8_fwd2d(const adct_plane* src, int32_t* coef, void* stream);

/* T8^T Y T8 for every block (block-major int32 in and out). */
int adct_t8_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream);

/* Single-pass 8x8 encoder with reconstruction, zonal form: Y stored to coef
 * unless NULL, the top-left r x r coefficients kept with S8 folded in
 * (r in [0, 8]), inverse, rounding and clamping into dst ([0, 255] for U8,
 * [-255, 255] for I16), and the exact per-image SSE when sse is non-NULL. */
int adct_t8_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                         int32_t image_height, int64_t* sse, void* stream);

/* Single-pass 8x8 encoder, quantised form: levels q = round(fp32(Y) * qs)
 * (half away from zero, saturated to int16) stored unless NULL, then
 * dequantisation to 6 fractional bits, inverse, rounding, clamping and the
 * optional SSE. */
int adct_t8_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst,
                         int32_t image_height, int64_t* sse, void* stream);

/* ---- the 32-point extension on 32x32 blocks ------------------------- */
/* Section 5 names 32- and 64-point extensions of the approach by the
 * scaled construction of its reference [Jridi2015] and prints no matrix;
 * these calls take the construction by which Section 2.1 builds T from two
 * 8-point blocks one level up:  T32 = P32 diag(T, T) B32, where B32 folds a
 * row into the sums x_j + x_{31-j} and differences x_j - x_{31-j}, T
 * (Section 2.1, 44 additions by Section 2.2) transforms each half, and P32
 * interleaves them (coefficient 2k from the sums, 2k + 1 from the
 * differences): 120 additions, entries in {0, +1, -1}, and T32 T32^T =
 * diag(2 d[u / 2]) with d the diagonal of T T^T.  The 32x32 codec mirrors
 * the 16-point one: S32 = diag(T32 T32^T)^(-1/2) folded into the zonal
 * weights W32 = 1024 / (d_u d_v) or the quantiser tables qs = fp32(s_u s_v
 * / Delta), dqs = fp32(1024 Delta s_u s_v); levels rounded half away from
 * zero and saturated to int16; reconstruction clamp(floor((R + 512) /
 * 1024)).  Planes: sides multiples of 32 (else ADCT_E_SHAPE), sample (0,0)
 * and the pitch 16-byte aligned (else ADCT_E_ALIGN); coefficient arrays are
 * block-major [nblk32][32][32], block k = by * (width/32) + bx, element
 * u*32 + v, 16-byte aligned; image_height a multiple of 32. */

/* Host copies of T32 (row-major), the diagonal of S32 and W32. */
int adct_t32_constants(int32_t* T1024, double* s32, int32_t* W1024);

/* Host copies of the 32x32 quantisation tables for `qp` in [0, 63]. */
int adct_t32_quant_tables(int qp, float* qs1024, float* dqs1024);

/* The kernels' 32-point butterflies run on the host with every addition
 * and subtraction counted (which = 0: T32, 1: T32^T); 32 values in and out. */
int adct_t32_host_butterfly_count(int32_t which, const int32_t* in32, int32_t* out32, int64_t* additions);

/* Y = T32 A T32^T for every 32x32 block A of src (U8 or I16); coef: device
 * int32 [nblk32][32][32]. */
int adct_t32_fwd2d(const adct_plane* src, int32_t* coef, void* stream);

/* T32^T Y T32 for every block (block-major int32 in and out). */
int adct_t32_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream);

/* Single-pass 32x32 encoder with reconstruction, zonal form: Y stored to
 * coef unless NULL, the top-left r x r coefficients kept with S32 folded in
 * (r in [0, 32]), inverse, rounding and clamping into dst ([0, 255] for U8,
 * [-255, 255] for I16), and the exact per-image SSE when sse is non-NULL. */
int adct_t32_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                          int32_t image_height, int64_t* sse, void* stream);

/* Single-pass 32x32 encoder, quantised form: levels stored unless NULL,
 * dequantisation to 10 fractional bits, inverse, rounding, clamping and the
 * optional SSE. */
int adct_t32_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst,
                          int32_t image_height, int64_t* sse, void* stream);

/* ---- the 64-point extension on 64x64 blocks ------------------------- */
/* The same construction one level further: T64 = P64 diag(T32, T32) B64,
 * B64 folding a row into the sums x_j + x_{63-j} and differences
 * x_j - x_{63-j}, T32 transforming each half and P64 interleaving them
 * (coefficient 2k from the sums, 2k + 1 from the differences): 304
 * additions, entries in {0, +1, -1}, and T64 T64^T = diag(2 d32[u / 2]),
 * entries 16, 32 or 64.  The 64x64 codec mirrors the 32x32 one with zonal
 * weights W64 = 4096 / (d_u d_v), quantiser tables qs = fp32(s_u s_v /
 * Delta), dqs = fp32(4096 Delta s_u s_v), levels rounded half away from
 * zero and saturated to int16, reconstruction clamp(floor((R + 2048) /
 * 4096)).  Planes: sides multiples of 64 (else ADCT_E_SHAPE), sample (0,0)
 * and the pitch 16-byte aligned (else ADCT_E_ALIGN), int16 samples within
 * [-2047, 2047]; coefficient arrays are block-major [nblk64][64][64], block
 * k = by * (width/64) + bx, element u*64 + v, 16-byte aligned; image_height
 * a multiple of 64. */

/* Host copies of T64 (row-major), the diagonal of S64 and W64. */
int adct_t64_constants(int32_t* T4096, double* s64, int32_t* W4096);

/* Host copies of the 64x64 quantisation tables for `qp` in [0, 63]. */
int adct_t64_quant_tables(int qp, float* qs4096, float* dqs4096);

/* The kernels' 64-point butterflies run on the host with every addition
 * and subtraction counted (which = 0: T64, 1: T64^T); 64 values in and out. */
int adct_t64_host_butterfly_count(int32_t which, const int32_t* in64, int32_t* out64, int64_t* additions);

/* Y = T64 A T64^T for every 64x64 block A of src (U8 or I16); coef: device
 * int32 [nblk64][64][64]. */
int adct_t64_fwd2d(const adct_plane* src, int32_t* coef, void* stream);

/* T64^T Y T64 for every block (block-major int32 in and out; exact while
 * every partial sum stays within int32, which holds for |Y| < 2^18). */
int adct_t64_inv2d(const int32_t* coef, int64_t nblk, int32_t* out, void* stream);

/* Single-pass 64x64 encoder with reconstruction, zonal form: Y stored to
 * coef unless NULL, the top-left r x r coefficients kept with S64 folded in
 * (r in [0, 64]), inverse, rounding and clamping into dst ([0, 255] for U8,
 * [-255, 255] for I16), and the exact per-image SSE when sse is non-NULL. */
int adct_t64_encode_zonal(const adct_plane* src, int r, int32_t* coef, const adct_plane* dst,
                          int32_t image_height, int64_t* sse, void* stream);

/* Single-pass 64x64 encoder, quantised form: levels stored unless NULL,
 * dequantisation to 12 fractional bits, inverse, rounding, clamping and the
 * optional SSE. */
int adct_t64_encode_quant(const adct_plane* src, int qp, int16_t* q, const adct_plane* dst,
                          int32_t image_height, int64_t* sse, void* stream);

/* ---- mixed 8/16-point coding ------------------------------------------ */
/* The codec of the second video scenario of Section 3.2, in which both the
 * 8-point (T8) and the 16-point (T) transforms are the approximations.  The
 * paper does not describe how the encoder picks a block's transform size;
 * here every 16x16 region is coded twice at the same QP, as one 16x16 block
 * (exactly as adct_encode_quant codes it) and as four 8x8 blocks (exactly
 * as adct_t8_encode_quant codes them), and keeps the coding with the lower
 * cost J = D + lambda * R, D the region's exact sum of squared
 * reconstruction errors and R its number of nonzero levels; equal costs
 * keep the 16x16 coding.  The decision is integer and exact.
 *
 * src, dst: planes as for adct_encode_quant (U8 or I16, sides multiples of
 * 16, same shape and type), dst receives the chosen reconstruction (clamped
 * to [0, 255] for U8, [-255, 255] for I16).
 * qp: [0, 63].  lambda: [0, ADCT_MIXED_MAX_LAMBDA] (else ADCT_E_ARG).
 * q: device int16 [nreg][16][16], 16-byte aligned, or NULL: the chosen levels
 *    of region k = by * (width/16) + bx, element u*16 + v; for a split
 *    region, 8x8 block (a, b) (a vertical) puts its element (i, j) at
 *    u = 8a + i, v = 8b + j.
 * split: device uint8 [nreg] or NULL: 1 where the region is coded as four
 *    8x8 blocks, else 0.
 * sse: device int64 [height / image_height] or NULL: per-image SSE of dst
 *    against src (image_height a multiple of 16 dividing the height).
 * Asynchronous on `stream`; allocates nothing. */
#define ADCT_MIXED_MAX_LAMBDA (((int64_t)1) << 40)
int adct_mixed_encode(const adct_plane* src, int qp, int64_t lambda, int16_t* q, uint8_t* split,
                      const adct_plane* dst, int32_t image_height, int64_t* sse, void* stream);

/* ---- image quality ----------------------------------------------------- */

/* Mean SSIM per image (the structural similarity index of Wang, Bovik,
 * Sheikh and Simoncelli, 2004, reported beside PSNR in Section 3.1): local
 * means, variances and covariance under an 11x11 Gaussian window of standard
 * deviation 1.5 (unit sum), K1 = 0.01, K2 = 0.03, L = 255, evaluated at every
 * position where the window lies inside the image, then averaged.  a, b:
 * uint8 planes of the same shape (else ADCT_E_DTYPE / ADCT_E_SHAPE), images
 * of `image_height` rows (a multiple of 16 dividing the height).
 * ssim: device float64 [height / image_height], 8-byte aligned, overwritten.
 * Computed in float64; the summation order over positions is not fixed, so
 * repeated calls agree to about 1e-15 relative.  ADCT_E_TOO_LARGE when the
 * planes hold more than 2^31 - 1 tiles of 16 x 48 positions. */
int adct_ssim(const adct_plane* a, const adct_plane* b, int32_t image_height, double* ssim, void* stream);

/* ---- uneven batches: one persistent launch over a device work queue -- */
/* Many images of different sizes coded by ONE launch: the host cuts every
 * image into items (runs of consecutive tiles that never span two images),
 * and persistent workgroups claim items from a device queue with one atomic
 * per claim until the queue is empty.  The reset of the queue and the launch
 * are captured once into a hipGraph that adct_batch_submit replays.
 * Per image the result is bit-identical to adct_encode_zonal /
 * adct_encode_quant on that image alone. */

typedef struct adct_job {
    adct_plane src;   /* input image, U8 or I16 (one type per batch)            */
    adct_plane dst;   /* reconstruction, same shape and type as src             */
    void* coef;       /* ADCT_OP_ZONAL, ADCT_OP_ZIGZAG: int32 coefficients;
                         ADCT_OP_QUANT: int16 levels; block-major
                         [nblk][16][16]; NULL: not stored                       */
    int64_t* sse;     /* device int64: exact SSE of dst against src, or NULL    */
} adct_job;

typedef struct adct_tune {
    int32_t tiles_per_group;  /* 8, 16 or 32 tiles transformed together by one
                                 workgroup of 8 threads per tile (1, 2 or 4
                                 wavefronts)                                   */
    int32_t groups_per_item;  /* tile groups per queue item, 1..64              */
    int32_t wgs_per_cu;       /* persistent workgroups per compute unit, 1..16  */
    int32_t reserved;
} adct_tune;

#define ADCT_OP_ZONAL  1  /* param = r in [0, 16]  (adct_encode_zonal per image)  */
#define ADCT_OP_QUANT  2  /* param = qp in [0, 63] (adct_encode_quant per image)  */
#define ADCT_OP_ZIGZAG 3  /* param = r in [0, 256] (adct_encode_zigzag per image) */

typedef struct adct_batch adct_batch;

/* The tuning used when none is given (host only). */
int adct_default_tune(adct_tune* out);

/* Host-side work-queue construction (no GPU needed): job j holds
 * tiles_per_job[j] tiles; items are written as triples (job, first tile,
 * tile count), each a run of at most tiles_per_group * groups_per_item
 * consecutive tiles of one job, in job order.  `items` holds room for
 * `capacity` triples; *n_items receives the count (ADCT_E_TOO_LARGE, with
 * *n_items set, when capacity is short; items may be NULL to count only). */
int adct_work_queue(const int64_t* tiles_per_job, int32_t njobs, int32_t tiles_per_group,
                    int32_t groups_per_item, uint32_t* items, int64_t capacity, int64_t* n_items);

/* Validates the jobs, builds the queue, uploads it and the job table to
 * library-owned device memory, and captures the graph (on the current
 * device).  `tune` NULL = adct_default_tune.  The job array is copied; the
 * buffers it points to stay owned by the caller and must outlive the batch.
 * Synchronous; ADCT_E_NOMEM / ADCT_E_HIP on allocation or runtime failure. */
int adct_batch_create(adct_batch** out, const adct_job* jobs, int32_t njobs, int32_t op, int32_t param,
                      const adct_tune* tune);

/* Replays the batch on `stream` (asynchronous).  Submissions of one batch on
 * different streams must not overlap: they share the queue. */
int adct_batch_submit(adct_batch* b, void* stream);

/* Tiles, queue items and the tuning of a batch (host). */
int adct_batch_info(const adct_batch* b, int64_t* tiles, int64_t* items, adct_tune* tune);

/* Releases the batch (synchronises its last submission first). */
int adct_batch_destroy(adct_batch* b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one uneven
 * batch coded like adct_batch_create + adct_batch_submit + adct_batch_destroy,
 * with identical results, but with no allocation and no graph.  The job
 * table, the work queue and the queue heads go into a static device array of
 * ADCT_NOALLOC_SCRATCH_BYTES that the library's code object holds on every
 * device it is loaded on, until the process ends; its address is looked up
 * once per device, on the first call there.  The host builds the queue and
 * copies the table and queue into the array with hipMemcpyAsync on `stream`
 * from host memory that it frees on return (HIP completes copies from
 * pageable memory before returning, so the call may wait for earlier work
 * on `stream`), then launches the reset kernel (queue heads and every job's
 * SSE cleared) and the persistent kernel on `stream` (current device).  The
 * caller's buffers must stay valid until the stream has run the launch.
 * Every call on one device shares that device's array and leaves the last
 * call's contents in it: calls that overlap on one device (different streams,
 * or host threads racing on one stream) race and give undefined results.
 * ADCT_E_TOO_LARGE when the table and queue exceed the array (fewer, larger
 * items -- a larger tiles_per_group * groups_per_item -- need less);
 * validation errors as adct_batch_create; nothing is launched on error.
 * `tune` NULL = adct_default_tune. */
#define ADCT_NOALLOC_SCRATCH_BYTES (16u << 20)
int adct_batch_run_noalloc(const adct_job* jobs, int32_t njobs, int32_t op, int32_t param, const adct_tune* tune,
                           void* stream);

/* Chooses a tuning for (op, param, these jobs) by timing every candidate
 * (tiles_per_group x groups_per_item x wgs_per_cu) `reps` times on the jobs
 * themselves -- their dst, coef and sse buffers are overwritten -- and keeps
 * the fastest.  When `cache_path` is non-NULL, a cached entry for the same
 * device architecture, compute-unit count, op, param and sample type is
 * returned without timing, and a new result is appended to the file (one
 * JSON object per line).  *ms (may be NULL) receives the chosen candidate's
 * median time, or -1 when it came from the cache.  Synchronous. */
int adct_autotune(int32_t op, int32_t param, const adct_job* jobs, int32_t njobs, const char* cache_path,
                  int32_t reps, adct_tune* out, double* ms);

/* ---- serving: continuous batching on a device-resident loop -------- */
/* Requests (uint8 images of any size that is a multiple of 16, each coded as
 * adct_encode_quant at the server's qp: levels and reconstruction kept on
 * the device, exact SSE reported) arrive over time.  A host thread admits
 * them in submission order when the server's device memory pool has room
 * (and fewer than max_inflight are held) and publishes each admitted request
 * to a persistent kernel through host-mapped memory.  One wave of that
 * kernel forwards new requests to its other workgroups, which claim work
 * items (runs of tiles of one request) as they appear, copy each item's
 * pixel rows from the caller's pinned host memory into the pool in long
 * contiguous runs and code them from there, so requests that arrive while
 * others run are coded alongside them; the last workgroup to finish a
 * request posts its SSE and a completion flag to host memory.  Requests of
 * at least dma_min_pixels pixels that arrive while others are in flight are
 * instead copied into the pool by the DMA engine, on a second stream, and
 * published once that copy is done, so that their transfer neither waits
 * for the loop's staging of the others nor holds it up (dma_policy).  In ADCT_SERVE_PLAIN mode the same
 * admission feeds a plain per-request path instead (one stream, first in
 * first out: copy in, adct_fwd2d_quant, adct_dequant_recon, SSE copy back,
 * event), the baseline the persistent loop is measured against.  In both
 * modes the host thread polls without sleeping while requests are
 * outstanding or the next one is due within 200 us (it then keeps one CPU
 * core busy).  While the persistent loop runs it occupies one hardware queue
 * of the device; work on another stream that the runtime maps to the same
 * queue waits until the loop ends (after idle_polls empty polls).  Results
 * are bit-identical between modes and between a request coded alone and in
 * any mix.  Times are in nanoseconds of the server clock (adct_now_ns). */

#define ADCT_SERVE_PERSISTENT 0
#define ADCT_SERVE_PLAIN      1

typedef struct adct_server_cfg {
    int64_t pool_bytes;      /* device pool for request data: 4 bytes per pixel
                                (the copied source, levels, reconstruction)      */
    int32_t qp;              /* quantiser for every request, [0, 63]            */
    int32_t mode;            /* ADCT_SERVE_PERSISTENT or ADCT_SERVE_PLAIN       */
    int32_t max_inflight;    /* admitted and not yet released, >= 1             */
    int32_t max_requests;    /* requests over the server's lifetime, >= 1       */
    int32_t auto_release;    /* 1: free a request's device data when it completes
                                (its SSE and times stay readable)               */
    int32_t tiles_per_item;  /* persistent: tiles per work item, a multiple of 16;
                                0 = per request: 16 for up to 2048 tiles, then
                                doubling up to 128 as the request grows          */
    int32_t wgs_per_cu;      /* persistent: loop workgroups per CU (0 = 2)      */
    int32_t idle_polls;      /* persistent: consecutive empty polls of the
                                dispatching wave (about 1-2 us each) before the
                                loop ends; the server relaunches it when work
                                reappears (0 = 100000)                           */
    int32_t dma_min_pixels;  /* persistent: requests of at least this many
                                pixels are "large"; a request copied into the
                                pool by the DMA engine (one copy on a second
                                stream) is published to the loop once the copy
                                is done, the others are staged by the loop.
                                0 = ADCT_SERVE_DMA_MIN_DEFAULT, -1 = no DMA      */
    int32_t dma_policy;      /* persistent: which requests go by DMA.
                                ADCT_SERVE_DMA_ADAPTIVE (0): a large request
                                when others are in flight (alone, the loop
                                stages it and codes while it crosses the link),
                                and a smaller one while the loop stages a large
                                one; ADCT_SERVE_DMA_BY_SIZE (1): every large
                                request                                          */
} adct_server_cfg;

#define ADCT_SERVE_DMA_MIN_DEFAULT (2048 * 2048)
#define ADCT_SERVE_DMA_ADAPTIVE 0
#define ADCT_SERVE_DMA_BY_SIZE  1

typedef struct adct_result {
    int32_t status;          /* ADCT_OK, ADCT_PENDING or ADCT_E_STOPPED          */
    int32_t height, width;
    int32_t reserved;
    void* dst;               /* device uint8 reconstruction [height][width]; NULL
                                once released                                    */
    void* q;                 /* device int16 levels [nblk][16][16]; NULL once released */
    int64_t sse;             /* exact SSE of dst against the submitted pixels    */
    int64_t t_arrival_ns;    /* when the request counts as arrived               */
    int64_t t_admit_ns;      /* when it got pool memory and its copy was issued  */
    int64_t t_done_ns;       /* when the server observed its completion          */
} adct_result;

typedef struct adct_stats {
    int64_t submitted, admitted, completed, cancelled;
    int64_t in_flight;       /* admitted and not yet completed                   */
    int64_t tiles_completed;
    int64_t pool_bytes, pool_high_water;
    double wall_s;           /* first arrival to last completion                 */
    double tiles_per_s;      /* tiles_completed / wall_s                         */
    double latency_p50_ms, latency_p99_ms, latency_mean_ms, latency_max_ms;
    double queue_p50_ms, queue_p99_ms;  /* arrival to admission                  */
    int64_t loop_launches;   /* persistent loop (re)launches                     */
    int64_t dma_copies;      /* persistent: requests copied into the pool by the
                                DMA engine (the rest were staged by the loop)    */
} adct_stats;

typedef struct adct_server adct_server;

/* Server clock (monotonic, ns). */
int64_t adct_now_ns(void);

/* Allocates the pool and the server's device state, starts its host thread
 * (and, in persistent mode, the device loop) on the current device. */
int adct_server_create(adct_server** out, const adct_server_cfg* cfg);

/* Queues one request.  host_pixels: uint8 [height][pitch_bytes] in host
 * memory, which must stay valid and unchanged until the request completes.
 * Persistent mode reads it from the device: it must be pinned memory the
 * device can address (hipHostMalloc, or a pinned torch tensor), else ADCT_E_ARG, with
 * host_pixels and pitch_bytes multiples of 16 (else ADCT_E_ALIGN).  Plain
 * mode copies it (pinned memory gives asynchronous copies).  arrival_ns < 0
 * means now; a later time holds the request back until then (open-loop
 * replay).  Requests are admitted in submission order.  ADCT_E_TOO_LARGE
 * when the request can never fit the pool or max_requests is used up. */
int adct_server_submit(adct_server* s, const void* host_pixels, int32_t height, int32_t width, int64_t pitch_bytes,
                       int64_t arrival_ns, uint64_t* ticket);

/* Non-blocking: ADCT_PENDING (> 0) until done, then ADCT_OK with *out
 * filled; ADCT_E_STOPPED for a cancelled request, ADCT_E_NOTFOUND for an
 * unknown ticket. */
int adct_server_poll(adct_server* s, uint64_t ticket, adct_result* out);

/* Blocks until every submitted request is done or cancelled, or until
 * timeout_ns passes (ADCT_E_TIMEOUT). */
int adct_server_wait_all(adct_server* s, int64_t timeout_ns);

/* Returns a completed request's device memory to the pool. */
int adct_server_release(adct_server* s, uint64_t ticket);

int adct_server_stats(adct_server* s, adct_stats* out);

/* drain = 1: finish every submitted request first; 0: cancel those not yet
 * admitted (admitted ones still finish).  Then stops the device loop. */
int adct_server_stop(adct_server* s, int32_t drain);

/* Stops (without draining) and frees everything. */
int adct_server_destroy(adct_server* s);

/* ---- the server's host policy, runnable without a GPU ------------------ */

/* Replays a sequence on the server's pool allocator (first fit, 256-byte
 * granules, coalescing) of the given capacity: ops[i] > 0 allocates that
 * many bytes (out[i] = offset or -1); ops[i] <= 0 frees the block allocated
 * by op -ops[i] (out[i] = 0).  *high_water (may be NULL) receives the peak
 * bytes in use.  ADCT_E_ARG for a free of an unknown block. */
int adct_pool_simulate(int64_t capacity, const int64_t* ops, int32_t nops, int64_t* out, int64_t* high_water);

/* Replays the server's admission rule (submission order, the head blocks
 * the rest; admitted when arrived, fewer than max_inflight held and the pool
 * can place it) on a fake clock: request i arrives at arrival[i], needs
 * bytes[i] and holds them for hold[i] after admission.  admit[i] receives
 * its admission time.  ADCT_E_TOO_LARGE when a request can never fit. */
int adct_admission_simulate(int64_t capacity, int32_t max_inflight, const int64_t* arrival, const int64_t* bytes,
                            const int64_t* hold, int32_t n, int64_t* admit);

/* Nearest-rank percentile p in [0, 100] of n values (the latency statistic
 * the server reports). */
int adct_percentile(const double* v, int64_t n, double p, double* out);

#ifdef __cplusplus
}
#endif

#endif /* ADCT_H */
