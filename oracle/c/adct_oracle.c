/*
 * Plain C oracle of the blockwise 2D 16-point approximate DCT.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite (checked against the
 * numpy oracle) and timed as the benchmark's CPU baseline.  Nothing in the
 * product path links or loads it, and it shares no code with the HIP
 * library.
 *
 * It is the plain definition, not a fast algorithm: per 16x16 block A,
 *   forward   Y = T A T^T                               (Section 3.1)
 *   zonal     Z' = (Y . mask_r) . W, W_uv = 256/(d_u d_v) (Section 3.1 with
 *             C-tilde = S T and S^2 = (T T^T)^-1, Section 2.1)
 *   inverse   R = T^T Z' T,  out = clamp(floor((R+128)/256), 0, 255)
 * as dense 16x16 matrix products in int64, parallel over blocks with OpenMP.
 */
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* T of Section 2.1, transcribed row by row. */
static const int64_t T[16][16] = {
    { 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    { 1, 1, 1, 1, 1, 1, 1, 1,-1,-1,-1,-1,-1,-1,-1,-1},
    { 1, 0, 0, 0, 0, 0, 0,-1,-1, 0, 0, 0, 0, 0, 0, 1},
    { 1, 1, 0, 0, 0, 0,-1,-1, 1, 1, 0, 0, 0, 0,-1,-1},
    { 1, 0, 0,-1,-1, 0, 0, 1, 1, 0, 0,-1,-1, 0, 0, 1},
    { 1, 1,-1,-1,-1,-1, 1, 1,-1,-1, 1, 1, 1, 1,-1,-1},
    { 0, 0,-1, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0,-1, 0, 0},
    { 0, 0, 0, 0, 0, 0,-1, 1,-1, 1, 0, 0, 0, 0, 0, 0},
    { 1,-1,-1, 1, 1,-1,-1, 1, 1,-1,-1, 1, 1,-1,-1, 1},
    { 0, 0,-1, 1, 0, 0, 0, 0, 0, 0, 0, 0,-1, 1, 0, 0},
    { 0,-1, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0,-1, 0},
    { 0, 0, 1, 1,-1,-1, 0, 0, 0, 0, 1, 1,-1,-1, 0, 0},
    { 0,-1, 1, 0, 0, 1,-1, 0, 0,-1, 1, 0, 0, 1,-1, 0},
    { 1,-1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1,-1},
    { 0, 0, 0,-1, 1, 0, 0, 0, 0, 0, 0, 1,-1, 0, 0, 0},
    { 0, 0, 0, 0,-1, 1, 0, 0, 0, 0,-1, 1, 0, 0, 0, 0},
};

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (timing at one thread and at all). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* coef[k][u][v] = sum_i sum_j T[u][i] A_k[i][j] T[v][j], raster block order. */
void oracle_fwd2d_u8(const uint8_t* img, int64_t H, int64_t W, int64_t pitch, int64_t* coef) {
    const int64_t bw = W / 16, nblk = (H / 16) * bw;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nblk; ++k) {
        const uint8_t* A = img + (k / bw) * 16 * pitch + (k % bw) * 16;
        int64_t P[16][16]; /* P = T A */
        for (int u = 0; u < 16; ++u)
            for (int j = 0; j < 16; ++j) {
                int64_t acc = 0;
                for (int i = 0; i < 16; ++i) acc += T[u][i] * (int64_t)A[i * pitch + j];
                P[u][j] = acc;
            }
        int64_t* Y = coef + k * 256;
        for (int u = 0; u < 16; ++u)
            for (int v = 0; v < 16; ++v) {
                int64_t acc = 0;
                for (int j = 0; j < 16; ++j) acc += P[u][j] * T[v][j];
                Y[u * 16 + v] = acc;
            }
    }
}

/* Zonal keep of the top-left r x r coefficients, weighted inverse, rounding
 * and clamping to uint8; sse[img] += sum (out - ref)^2 per image of
 * image_h rows (sse may be NULL). */
void oracle_zonal_recon_u8(const int64_t* coef, int64_t H, int64_t W, int r,
                           uint8_t* out, int64_t pitch, const uint8_t* ref,
                           int64_t image_h, int64_t* sse) {
    int64_t d[16];
    for (int u = 0; u < 16; ++u) {
        d[u] = 0;
        for (int j = 0; j < 16; ++j) d[u] += T[u][j] * T[u][j];
    }
    const int64_t bw = W / 16, nblk = (H / 16) * bw;
    const int64_t nimg = sse ? H / image_h : 0;
    if (sse) memset(sse, 0, sizeof(int64_t) * (size_t)nimg);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nblk; ++k) {
        const int64_t* Y = coef + k * 256;
        int64_t Z[16][16], Q[16][16];
        for (int u = 0; u < 16; ++u)
            for (int v = 0; v < 16; ++v)
                Z[u][v] = (u < r && v < r) ? Y[u * 16 + v] * (256 / (d[u] * d[v])) : 0;
        for (int i = 0; i < 16; ++i) /* Q = T^T Z */
            for (int v = 0; v < 16; ++v) {
                int64_t acc = 0;
                for (int u = 0; u < 16; ++u) acc += T[u][i] * Z[u][v];
                Q[i][v] = acc;
            }
        const int64_t y0 = (k / bw) * 16, x0 = (k % bw) * 16;
        int64_t local = 0;
        for (int i = 0; i < 16; ++i)
            for (int j = 0; j < 16; ++j) {
                int64_t R = 0; /* R = Q T */
                for (int v = 0; v < 16; ++v) R += Q[i][v] * T[v][j];
                int64_t o = R + 128;
                o = (o >= 0) ? o / 256 : -((-o + 255) / 256); /* floor division */
                if (o < 0) o = 0;
                if (o > 255) o = 255;
                out[(y0 + i) * pitch + x0 + j] = (uint8_t)o;
                if (ref) {
                    int64_t e = o - (int64_t)ref[(y0 + i) * pitch + x0 + j];
                    local += e * e;
                }
            }
        if (sse) {
#pragma omp atomic
            sse[y0 / image_h] += local;
        }
    }
}
