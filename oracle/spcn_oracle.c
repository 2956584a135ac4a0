/*
 * spcn_oracle.c -- FP64 CPU oracle for SPCN.  TEST INFRASTRUCTURE ONLY (see spcn_oracle.h).
 *
 * Plain, slow and obviously correct by construction: every step is the paper's definition written
 * out in double precision, with no blocking, fusion or reordering beyond what that definition says.
 * Built with -O2 -fno-fast-math -ffp-contract=off so that no multiply-add is contracted.
 */
#include "spcn_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Eq. (1), Sec. 2.1 step 1 --- */

/* v = log(i0 / i).  Readings: an intensity of 0 has no finite OD and is read as 1; an intensity
 * above i0 (possible once i0 is estimated per channel, Sec. 3.1 item 1) gives OD 0, not < 0. */
double orc_od_u8(double i0, int intensity) {
    double i = intensity < 1 ? 1.0 : (double)intensity;
    double v = log(i0 / i);
    return v > 0.0 ? v : 0.0;
}

/* Float pixels in [0,1] are 8-bit intensities divided by 255, so the smallest meaningful value is
 * 1/255; values below it are read as 1/255 (same reading as intensity 0 above). */
double orc_od_f(double i0, double x) {
    double lo = 1.0 / 255.0;
    double xi = x < lo ? lo : x;
    double v = log(i0 / xi);
    return v > 0.0 ? v : 0.0;
}

/* ------------------------------------------------ Eq. (2) with W fixed, Sec. 2.1 step 2 ------- */

/* Objective of Eq. (2) for one pixel, without the constant ||v||^2:
 *   phi(h) = ||v - W h||^2 - ||v||^2 + lambda (h0 + h1).
 * Computed literally from the residual so that the comparison below is the definition itself. */
static double pixel_objective(const double W[6], double lambda, const double v[3], const double h[2]) {
    double r2 = 0.0, v2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double r = v[c] - (W[c] * h[0] + W[c + 3] * h[1]);
        r2 += r * r;
        v2 += v[c] * v[c];
    }
    return (r2 - v2) + lambda * (h[0] + h[1]);
}

int orc_solve_pixel(const double W[6], double lambda, const double v[3], double h[2]) {
    /* Normal-equation quantities: G = W^T W and b = W^T v - lambda/2 (Eq. 2 as printed, without the
     * factor 1/2 on the squared norm, so the gradient of the penalty is lambda, i.e. lambda/2 after
     * dividing the stationarity condition by 2). */
    double g00 = 0, g01 = 0, g11 = 0, b0 = 0, b1 = 0;
    for (int c = 0; c < 3; ++c) {
        g00 += W[c] * W[c];
        g01 += W[c] * W[c + 3];
        g11 += W[c + 3] * W[c + 3];
        b0 += W[c] * v[c];
        b1 += W[c + 3] * v[c];
    }
    b0 -= 0.5 * lambda;
    b1 -= 0.5 * lambda;

    /* The minimiser over the closed quadrant lies on one of its four faces; on each face it is the
     * minimiser of the restricted convex quadratic.  Enumerate the four and keep the best. */
    double cand[4][2];
    int valid[4] = {1, 1, 1, 0};
    cand[0][0] = 0.0; cand[0][1] = 0.0;                                   /* origin           */
    cand[1][0] = g00 > 0.0 ? fmax(0.0, b0 / g00) : 0.0; cand[1][1] = 0.0;  /* edge h1 = 0      */
    cand[2][0] = 0.0; cand[2][1] = g11 > 0.0 ? fmax(0.0, b1 / g11) : 0.0;  /* edge h0 = 0      */
    double det = g00 * g11 - g01 * g01;                                   /* interior: G h = b */
    if (det > 0.0) {
        cand[3][0] = (g11 * b0 - g01 * b1) / det;
        cand[3][1] = (g00 * b1 - g01 * b0) / det;
        valid[3] = cand[3][0] >= 0.0 && cand[3][1] >= 0.0;
    }
    int best = 0;
    double best_obj = pixel_objective(W, lambda, v, cand[0]);
    for (int k = 1; k < 4; ++k) {
        if (!valid[k]) continue;
        double o = pixel_objective(W, lambda, v, cand[k]);
        if (o < best_obj) { best_obj = o; best = k; }   /* exact ties keep the lower index */
    }
    h[0] = cand[best][0];
    h[1] = cand[best][1];
    return best;
}

/* ----------------------------------------------------- non-white mask, Sec. 3.1 item 2 -------- */

/* "Non-white" is read as mean intensity below 220, i.e. R + G + B < 660 (white_sum), in integers. */
int orc_is_tissue_u8(const uint8_t* px, int white_sum) {
    if (white_sum <= 0) return 1;
    int s = (int)px[0] + (int)px[1] + (int)px[2];
    return s < white_sum;
}

int orc_is_tissue_f32(float x0, float x1, float x2, int white_sum) {
    if (white_sum <= 0) return 1;
    volatile float s = x0 + x1;   /* volatile: keep every FP32 rounding exactly as stated */
    s = s + x2;
    volatile float t = s * 255.0f;
    return t < (float)white_sum;
}

void orc_densities_u8(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                      double lambda, int white_sum, double* H, uint8_t* mask) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_px; ++i) {
        const uint8_t* px = img + 3 * i;
        double v[3], h[2];
        for (int c = 0; c < 3; ++c) v[c] = orc_od_u8(i0[c], px[c]);
        orc_solve_pixel(W, lambda, v, h);
        H[i] = h[0];
        H[n_px + i] = h[1];
        if (mask) mask[i] = (uint8_t)orc_is_tissue_u8(px, white_sum);
    }
}

/* ------------------------------------------------- percentile of Eq. (3), Sec. 2.1 step 3 ----- */

/* Histogram over tissue pixels: bin k covers [k, k+1) * hist_hi / bins; values at or above the
 * top edge land in the last bin. */
void orc_histogram(const double* H, const uint8_t* mask, int64_t n_px, const double hist_hi[2],
                   int bins, uint64_t* hist) {
    memset(hist, 0, sizeof(uint64_t) * 2 * (size_t)bins);
    for (int j = 0; j < 2; ++j) {
        double width = hist_hi[j] / bins;
        for (int64_t i = 0; i < n_px; ++i) {
            if (mask && !mask[i]) continue;
            double f = floor(H[j * n_px + i] / width);
            int64_t k = f > (double)(bins - 1) ? bins - 1 : (int64_t)f;
            if (k < 0) k = 0;
            hist[j * bins + k] += 1;
        }
    }
}

/* Percentile q (a fraction) of the n counted values, linear inside the bin where the cumulative
 * count first reaches q*n (the histogram's own CDF, piecewise linear). */
int orc_percentile_hist(const uint64_t* counts, int bins, double hist_hi, double q, double* P, int* kstar) {
    uint64_t n = 0;
    for (int k = 0; k < bins; ++k) n += counts[k];
    if (n == 0) { *P = 0.0; if (kstar) *kstar = -1; return ORC_NO_TISSUE; }
    double r = q * (double)n;
    uint64_t below = 0;
    int k = 0;
    while ((double)(below + counts[k]) < r) { below += counts[k]; ++k; }
    double width = hist_hi / bins;
    *P = width * ((double)k + (r - (double)below) / (double)counts[k]);
    if (kstar) *kstar = k;
    int flags = ORC_OK;
    if (k == bins - 1) flags |= ORC_RANGE;
    if (k == 0) flags |= ORC_BIN0;
    return flags;
}

/* One retry of the histogram range: count at hist_hi, and double the range of each stain whose
 * percentile lands in the last bin (while that range is below 256). */
int orc_settle_range(const double* H, const uint8_t* mask, int64_t n_px, const double hist_hi[2], int bins,
                     double q, double range_out[2]) {
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (size_t)bins);
    orc_histogram(H, mask, n_px, hist_hi, bins, hist);
    int bits = 0;
    for (int j = 0; j < 2; ++j) {
        double P;
        int k;
        orc_percentile_hist(hist + j * bins, bins, hist_hi[j], q, &P, &k);
        range_out[j] = hist_hi[j];
        if (k == bins - 1 && hist_hi[j] < 256.0) {
            range_out[j] = 2.0 * hist_hi[j];
            bits |= 1 << j;
        }
    }
    free(hist);
    return bits;
}

static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

int orc_percentile_exact(const double* h, const uint8_t* mask, int64_t n_px, double q, double* P, int64_t* idx) {
    int64_t n = 0;
    for (int64_t i = 0; i < n_px; ++i) n += (!mask || mask[i]) ? 1 : 0;
    if (n == 0) { *P = 0.0; if (idx) *idx = -1; return ORC_NO_TISSUE; }
    double* vals = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t m = 0;
    for (int64_t i = 0; i < n_px; ++i) if (!mask || mask[i]) vals[m++] = h[i];
    qsort(vals, (size_t)n, sizeof(double), cmp_double);
    int64_t k = (int64_t)ceil(q * (double)n);
    if (k < 1) k = 1;
    if (k > n) k = n;
    *P = vals[k - 1];
    free(vals);
    if (idx) {
        *idx = -1;
        for (int64_t i = 0; i < n_px; ++i)
            if ((!mask || mask[i]) && h[i] == *P) { *idx = i; break; }
    }
    return ORC_OK;
}

/* ------------------------------------------------------ Eqs. (3)-(4), Sec. 2.1 steps 3-4 ------ */

/* Eq. (3): v'_c = sum_j W_tgt[c,j] * s_j * h_j with s_j = P99_tgt,j / P99_src,j;
 * Eq. (4): y_c = i0_out,c * exp(-v'_c). */
void orc_reconstruct_pixel(const double h[2], const double W_tgt[6], const double s[2],
                           const double i0_out[3], double y[3]) {
    for (int c = 0; c < 3; ++c) {
        double vp = W_tgt[c] * (s[0] * h[0]) + W_tgt[c + 3] * (s[1] * h[1]);
        y[c] = i0_out[c] * exp(-vp);
    }
}

/* Scale of Eq. (3) from the two percentiles; an absent stain (P in bin 0), no tissue or a
 * non-positive P keeps the stain's density unscaled (s = 1). */
static double stain_scale(double scale_tgt, double P, int flags) {
    if ((flags & (ORC_NO_TISSUE | ORC_BIN0)) || !(P > 0.0)) return 1.0;
    return scale_tgt / P;
}

int orc_normalize_u8(const uint8_t* src, int64_t n_px, const double W_src[6], const double W_tgt[6],
                     const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                     double lambda, int white_sum, double q, const double hist_hi[2], int bins,
                     uint8_t* out, double* stats, uint64_t* hist_out) {
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n_px);
    uint8_t* mask = (uint8_t*)malloc((size_t)n_px);
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (size_t)bins);
    orc_densities_u8(src, n_px, W_src, i0_in, lambda, white_sum, H, mask);
    orc_histogram(H, mask, n_px, hist_hi, bins, hist);
    double P[2], s[2];
    int flags[2], all = 0;
    for (int j = 0; j < 2; ++j) {
        flags[j] = orc_percentile_hist(hist + j * bins, bins, hist_hi[j], q, &P[j], NULL);
        s[j] = stain_scale(scale_tgt[j], P[j], flags[j]);
        all |= flags[j];
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_px; ++i) {
        double h[2] = {H[i], H[n_px + i]}, y[3];
        orc_reconstruct_pixel(h, W_tgt, s, i0_out, y);
        for (int c = 0; c < 3; ++c) {
            double r = nearbyint(y[c]);            /* round half to even */
            r = r < 0.0 ? 0.0 : (r > 255.0 ? 255.0 : r);
            out[3 * i + c] = (uint8_t)r;
        }
    }
    if (stats) {
        uint64_t n = 0;
        for (int k = 0; k < bins; ++k) n += hist[k];
        stats[0] = P[0]; stats[1] = P[1]; stats[2] = s[0]; stats[3] = s[1];
        stats[4] = flags[0]; stats[5] = flags[1]; stats[6] = (double)n; stats[7] = 0.0;
    }
    if (hist_out) memcpy(hist_out, hist, sizeof(uint64_t) * 2 * (size_t)bins);
    free(H); free(mask); free(hist);
    return all;
}

void orc_recolor_u8(const uint8_t* src, int64_t n_px, const double W_src[6], const double W_tgt[6],
                    const double scale_tgt[2], const double P_src[2], const double i0_in[3],
                    const double i0_out[3], double lambda, int white_sum, uint8_t* out) {
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n_px);
    uint8_t* mask = (uint8_t*)malloc((size_t)n_px);
    orc_densities_u8(src, n_px, W_src, i0_in, lambda, white_sum, H, mask);
    double s[2];
    for (int j = 0; j < 2; ++j) s[j] = stain_scale(scale_tgt[j], P_src[j], ORC_OK);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_px; ++i) {
        double h[2] = {H[i], H[n_px + i]}, y[3];
        orc_reconstruct_pixel(h, W_tgt, s, i0_out, y);
        for (int c = 0; c < 3; ++c) {
            double r = nearbyint(y[c]);
            r = r < 0.0 ? 0.0 : (r > 255.0 ? 255.0 : r);
            out[3 * i + c] = (uint8_t)r;
        }
    }
    free(H); free(mask);
}

int orc_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const double W[6],
                         const double i0[3], double lambda, int white_sum, double q,
                         const double hist_hi[2], int bins, int64_t band_rows, double* band_P,
                         int* band_flags, double median_P[2]) {
    int64_t n_bands = (height + band_rows - 1) / band_rows;
    double* P = (double*)malloc(sizeof(double) * 2 * (size_t)n_bands);
    int* F = (int*)malloc(sizeof(int) * 2 * (size_t)n_bands);
    uint64_t* hist = (uint64_t*)malloc(sizeof(uint64_t) * 2 * (size_t)bins);
    for (int64_t b = 0; b < n_bands; ++b) {
        int64_t r0 = b * band_rows, r1 = r0 + band_rows < height ? r0 + band_rows : height;
        int64_t n = (r1 - r0) * width;
        double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n);
        uint8_t* mask = (uint8_t*)malloc((size_t)n);
        orc_densities_u8(img + 3 * r0 * width, n, W, i0, lambda, white_sum, H, mask);
        orc_histogram(H, mask, n, hist_hi, bins, hist);
        for (int j = 0; j < 2; ++j)
            F[2 * b + j] = orc_percentile_hist(hist + j * bins, bins, hist_hi[j], q, &P[2 * b + j], NULL);
        free(H); free(mask);
    }
    int flags = ORC_OK;
    double* vals = (double*)malloc(sizeof(double) * (size_t)n_bands);
    for (int j = 0; j < 2; ++j) {
        int64_t m = 0;
        for (int64_t b = 0; b < n_bands; ++b)
            if (!(F[2 * b + j] & ORC_NO_TISSUE)) vals[m++] = P[2 * b + j];
        if (m == 0) { median_P[j] = 0.0; flags |= ORC_NO_TISSUE; continue; }
        qsort(vals, (size_t)m, sizeof(double), cmp_double);
        median_P[j] = (m & 1) ? vals[m / 2] : 0.5 * (vals[m / 2 - 1] + vals[m / 2]);
    }
    if (band_P) memcpy(band_P, P, sizeof(double) * 2 * (size_t)n_bands);
    if (band_flags) memcpy(band_flags, F, sizeof(int) * 2 * (size_t)n_bands);
    free(vals); free(P); free(F); free(hist);
    return flags;
}

/* ------------------------------------------- basis estimation, Eq. (2), Sec. 3.1-3.2 ---------- */

uint64_t orc_splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int64_t orc_sample_tissue(const uint8_t* img, int64_t n_px, int white_sum, uint64_t seed,
                          int64_t n_s, int64_t max_cand, int64_t* idx_out) {
    int64_t kept = 0;
    for (int64_t t = 0; t < max_cand && kept < n_s; ++t) {
        uint64_t r = orc_splitmix64(seed, (uint64_t)t);
        int64_t i = (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)n_px) >> 64);
        if (orc_is_tissue_u8(img + 3 * i, white_sum)) idx_out[kept++] = i;
    }
    return kept;
}

int orc_sample_percentile(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                          double lambda, int white_sum, uint64_t seed, int64_t n_s, int64_t max_cand,
                          double q, double P[2], int64_t* kept) {
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_s > 0 ? n_s : 1));
    int64_t n = orc_sample_tissue(img, n_px, white_sum, seed, n_s, max_cand, idx);
    if (kept) *kept = n;
    if (n == 0) { P[0] = P[1] = 0.0; free(idx); return ORC_NO_TISSUE; }
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        const uint8_t* p = img + 3 * idx[i];
        double v[3], h[2];
        for (int c = 0; c < 3; ++c) v[c] = orc_od_u8(i0[c], p[c]);
        orc_solve_pixel(W, lambda, v, h);
        H[i] = h[0]; H[n + i] = h[1];
    }
    for (int j = 0; j < 2; ++j) orc_percentile_exact(H + j * n, NULL, n, q, &P[j], NULL);
    free(H); free(idx);
    return ORC_OK;
}

int orc_exact_percentile_u8(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                            double lambda, int white_sum, double q, double P[2], int64_t* n_tissue) {
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)(n_px > 0 ? n_px : 1));
    uint8_t* mask = (uint8_t*)malloc((size_t)(n_px > 0 ? n_px : 1));
    orc_densities_u8(img, n_px, W, i0, lambda, white_sum, H, mask);
    int64_t n = 0;
    for (int64_t i = 0; i < n_px; ++i) n += mask[i];
    if (n_tissue) *n_tissue = n;
    int flags = ORC_OK;
    for (int j = 0; j < 2; ++j) flags |= orc_percentile_exact(H + j * n_px, mask, n_px, q, &P[j], NULL);
    free(H); free(mask);
    return flags;
}

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

int64_t orc_estimate_i0(const uint8_t* img, int64_t n_px, int white_sum, uint64_t seed, int64_t n_s,
                        int64_t max_cand, double q, double i0_out[3]) {
    int* vals[3];
    for (int c = 0; c < 3; ++c) vals[c] = (int*)malloc(sizeof(int) * (size_t)(n_s > 0 ? n_s : 1));
    int64_t kept = 0;
    for (int64_t t = 0; t < max_cand && kept < n_s; ++t) {
        uint64_t r = orc_splitmix64(seed, (uint64_t)t);
        int64_t i = (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)n_px) >> 64);
        const uint8_t* p = img + 3 * i;
        if ((int)p[0] + (int)p[1] + (int)p[2] > white_sum) {
            for (int c = 0; c < 3; ++c) vals[c][kept] = p[c];
            ++kept;
        }
    }
    if (kept > 0) {
        int64_t k = (int64_t)ceil(q * (double)kept);
        if (k < 1) k = 1;
        if (k > kept) k = kept;
        for (int c = 0; c < 3; ++c) {
            qsort(vals[c], (size_t)kept, sizeof(int), cmp_int);
            i0_out[c] = (double)vals[c][k - 1];
        }
    }
    for (int c = 0; c < 3; ++c) free(vals[c]);
    return kept;
}

double orc_nmf_objective(const double* V, const double* H, int64_t n, const double W[6], double lambda) {
    double f = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) {
            double r = V[c * n + i] - (W[c] * H[i] + W[c + 3] * H[n + i]);
            f += r * r;
        }
        f += lambda * (H[i] + H[n + i]);
    }
    return f;
}

int orc_stain_order_swap(const double W[6]) {
    /* hematoxylin is the stain whose OD is larger in red than in blue by the most */
    double d0 = W[0] - W[2], d1 = W[3] - W[5];
    return d1 > d0;
}

static void h_step(const double* V, int64_t n, const double W[6], double lambda, double* H) {
    for (int64_t i = 0; i < n; ++i) {
        double v[3] = {V[i], V[n + i], V[2 * n + i]}, h[2];
        orc_solve_pixel(W, lambda, v, h);
        H[i] = h[0];
        H[n + i] = h[1];
    }
}

void orc_nmf(const double* V, int64_t n, double lambda, int T, double W_io[6],
             double* obj_trace, double q, double* sample_p99) {
    double W[6];
    memcpy(W, W_io, sizeof W);
    double* H = (double*)calloc(2 * (size_t)(n > 0 ? n : 1), sizeof(double));
    for (int t = 0; t < T; ++t) {
        /* H-step: Eq. (2) is separable over pixels once W is fixed; each pixel is solved exactly. */
        h_step(V, n, W, lambda, H);
        if (obj_trace) obj_trace[2 * t] = orc_nmf_objective(V, H, n, W, lambda);
        /* W-step: one pass of block-coordinate descent over the two columns.  With A = H H^T and
         * B = V H^T, the squared error restricted to column j is A_jj ||w_j - u||^2 + const with
         * u = w_j + (B_j - W A_j) / A_jj; its minimiser over {w >= 0, ||w|| <= 1} is the Euclidean
         * projection of u, i.e. max(u, 0) rescaled onto the ball if it lies outside.  The unit-norm
         * equality of Eq. (2) is restored after the last iteration. */
        double A[2][2] = {{0, 0}, {0, 0}}, B[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t i = 0; i < n; ++i) {
            double h0 = H[i], h1 = H[n + i];
            A[0][0] += h0 * h0; A[0][1] += h0 * h1; A[1][1] += h1 * h1;
            for (int c = 0; c < 3; ++c) { B[c][0] += V[c * n + i] * h0; B[c][1] += V[c * n + i] * h1; }
        }
        A[1][0] = A[0][1];
        for (int j = 0; j < 2; ++j) {
            if (!(A[j][j] > 0.0)) continue;            /* stain unused by every sample: keep w_j */
            double u[3], nrm2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                double WAj = W[c] * A[0][j] + W[c + 3] * A[1][j];
                u[c] = W[c + 3 * j] + (B[c][j] - WAj) / A[j][j];
                if (u[c] < 0.0) u[c] = 0.0;
                nrm2 += u[c] * u[c];
            }
            if (!(nrm2 > 0.0)) continue;               /* projection is the zero vector: keep w_j */
            double scale = nrm2 > 1.0 ? 1.0 / sqrt(nrm2) : 1.0;
            for (int c = 0; c < 3; ++c) W[c + 3 * j] = u[c] * scale;
        }
        if (obj_trace) obj_trace[2 * t + 1] = orc_nmf_objective(V, H, n, W, lambda);
    }
    for (int j = 0; j < 2; ++j) {
        double nrm = sqrt(W[3 * j] * W[3 * j] + W[3 * j + 1] * W[3 * j + 1] + W[3 * j + 2] * W[3 * j + 2]);
        if (nrm > 0.0) for (int c = 0; c < 3; ++c) W[c + 3 * j] /= nrm;
    }
    if (orc_stain_order_swap(W)) {
        for (int c = 0; c < 3; ++c) { double t = W[c]; W[c] = W[c + 3]; W[c + 3] = t; }
    }
    if (sample_p99) {
        h_step(V, n, W, lambda, H);
        for (int j = 0; j < 2; ++j) {
            double P = 0.0;
            if (n > 0) orc_percentile_exact(H + j * n, NULL, n, q, &P, NULL);
            sample_p99[j] = P;
        }
    }
    memcpy(W_io, W, sizeof W);
    free(H);
}

/* ----------------------------------------------- differentiable float path (extension) -------- */

static void f32_densities(const double* x, int64_t n_px, const double W_src[6], const double i0_in[3],
                          double lambda, int white_sum, double* H, uint8_t* mask) {
    for (int64_t i = 0; i < n_px; ++i) {
        double v[3], h[2];
        for (int c = 0; c < 3; ++c) v[c] = orc_od_f(i0_in[c], x[c * n_px + i]);
        orc_solve_pixel(W_src, lambda, v, h);
        H[i] = h[0];
        H[n_px + i] = h[1];
        mask[i] = (uint8_t)orc_is_tissue_f32((float)x[i], (float)x[n_px + i], (float)x[2 * n_px + i], white_sum);
    }
}

int orc_forward_f32(const double* x, int64_t n_px, const double W_src[6], const double W_tgt[6],
                    const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                    double lambda, int white_sum, double q, double* y, double* P, int64_t* istar,
                    double* H_out) {
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n_px);
    uint8_t* mask = (uint8_t*)malloc((size_t)n_px);
    f32_densities(x, n_px, W_src, i0_in, lambda, white_sum, H, mask);
    int flags = 0;
    double s[2];
    for (int j = 0; j < 2; ++j) {
        int f = orc_percentile_exact(H + j * n_px, mask, n_px, q, &P[j], &istar[j]);
        if (f == ORC_OK && !(P[j] > 0.0)) f = ORC_BIN0;
        s[j] = stain_scale(scale_tgt[j], P[j], f);
        flags |= f;
    }
    for (int64_t i = 0; i < n_px; ++i) {
        double h[2] = {H[i], H[n_px + i]}, yy[3];
        orc_reconstruct_pixel(h, W_tgt, s, i0_out, yy);
        for (int c = 0; c < 3; ++c) y[c * n_px + i] = yy[c];
    }
    if (H_out) memcpy(H_out, H, sizeof(double) * 2 * (size_t)n_px);
    free(H); free(mask);
    return flags;
}

/* Distance of each pixel of a float image from a change of its active set in Eq. (2) (W fixed):
 * the smallest magnitude among the quantities whose signs pick the face of the quadrant that holds
 * the minimiser -- the one-stain minimisers b_j / g_jj and, when G is regular, the two entries of
 * G^-1 b.  A pixel whose margin is tiny may be solved on another face in FP32 than in FP64.  (The
 * OD clamps of Eq. (1) and the non-white mask are decided on the same FP32 input on both sides and
 * are not counted.) */
void orc_active_margin_f32(const double* x, int64_t n_px, const double W[6], const double i0_in[3],
                           double lambda, double* margin) {
    double g00 = 0, g01 = 0, g11 = 0;
    for (int c = 0; c < 3; ++c) {
        g00 += W[c] * W[c]; g01 += W[c] * W[c + 3]; g11 += W[c + 3] * W[c + 3];
    }
    double det = g00 * g11 - g01 * g01;
    for (int64_t i = 0; i < n_px; ++i) {
        double v[3], b0 = 0.0, b1 = 0.0, m = INFINITY;
        for (int c = 0; c < 3; ++c) {
            v[c] = orc_od_f(i0_in[c], x[c * n_px + i]);
            b0 += W[c] * v[c];
            b1 += W[c + 3] * v[c];
        }
        b0 -= 0.5 * lambda;
        b1 -= 0.5 * lambda;
        if (g00 > 0.0) m = fmin(m, fabs(b0 / g00));
        if (g11 > 0.0) m = fmin(m, fabs(b1 / g11));
        if (det > 0.0) {
            m = fmin(m, fabs((g11 * b0 - g01 * b1) / det));
            m = fmin(m, fabs((g00 * b1 - g01 * b0) / det));
        }
        margin[i] = m;
    }
}

/* Adjoint, derived by hand from the forward definitions above:
 *   y_c = i0_out,c exp(-u_c),  u_c = sum_j Wt[c,j] s_j h_j,  s_j = S_j / P_j,  P_j = h_j(pixel i*_j).
 *   ubar_c = -y_c gbar_c;  dWt[c,j] = sum_i ubar_ic s_j h_ij;  ds_j = sum_i sum_c ubar_ic Wt[c,j] h_ij;
 *   dS_j = ds_j / P_j;  Pbar_j = -(s_j / P_j) ds_j, added to hbar at pixel i*_j;
 *   hbar_ij = s_j sum_c Wt[c,j] ubar_ic.
 * Per pixel, on the active set F = {j : h_j > 0} the solution satisfies G_FF h_F = b_F with
 * b = W^T v - lambda/2, so vbar = W_F G_FF^{-1} hbar_F; finally dv_c/dx_c = -1/x_c where the OD
 * is neither clamped at 1/255 nor at 0. */
int orc_backward_f32(const double* x, int64_t n_px, const double W_src[6], const double W_tgt[6],
                     const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                     double lambda, int white_sum, double q, const double* grad_y,
                     const int64_t* istar_in, double* grad_x, double grad_W_tgt[6],
                     double grad_scale[2]) {
    double* H = (double*)malloc(sizeof(double) * 2 * (size_t)n_px);
    uint8_t* mask = (uint8_t*)malloc((size_t)n_px);
    f32_densities(x, n_px, W_src, i0_in, lambda, white_sum, H, mask);
    double P[2], s[2];
    int64_t istar[2];
    int fl[2], flags = 0;
    for (int j = 0; j < 2; ++j) {
        fl[j] = orc_percentile_exact(H + j * n_px, mask, n_px, q, &P[j], &istar[j]);
        if (fl[j] == ORC_OK && !(P[j] > 0.0)) fl[j] = ORC_BIN0;
        if (istar_in && fl[j] == ORC_OK) { istar[j] = istar_in[j]; P[j] = H[j * n_px + istar[j]]; }
        s[j] = stain_scale(scale_tgt[j], P[j], fl[j]);
        flags |= fl[j];
    }
    double* hbar = (double*)calloc(2 * (size_t)n_px, sizeof(double));
    double dW[6] = {0, 0, 0, 0, 0, 0}, ds[2] = {0, 0};
    for (int64_t i = 0; i < n_px; ++i) {
        double h[2] = {H[i], H[n_px + i]}, y[3], ub[3];
        orc_reconstruct_pixel(h, W_tgt, s, i0_out, y);
        for (int c = 0; c < 3; ++c) ub[c] = -y[c] * grad_y[c * n_px + i];
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int c = 0; c < 3; ++c) {
                dW[c + 3 * j] += ub[c] * s[j] * h[j];
                acc += W_tgt[c + 3 * j] * ub[c];
            }
            ds[j] += acc * h[j];
            hbar[j * n_px + i] = s[j] * acc;
        }
    }
    for (int j = 0; j < 2; ++j) {
        int scaled = !(fl[j] & (ORC_NO_TISSUE | ORC_BIN0));
        grad_scale[j] = scaled ? ds[j] / P[j] : 0.0;
        if (scaled) hbar[j * n_px + istar[j]] += -(s[j] / P[j]) * ds[j];
    }
    double g00 = 0, g01 = 0, g11 = 0;
    for (int c = 0; c < 3; ++c) {
        g00 += W_src[c] * W_src[c]; g01 += W_src[c] * W_src[c + 3]; g11 += W_src[c + 3] * W_src[c + 3];
    }
    double det = g00 * g11 - g01 * g01;
    for (int64_t i = 0; i < n_px; ++i) {
        double hb0 = hbar[i], hb1 = hbar[n_px + i];
        int a0 = H[i] > 0.0, a1 = H[n_px + i] > 0.0;
        double z0 = 0.0, z1 = 0.0;                    /* z = G_FF^{-1} hbar_F, zero off F */
        if (a0 && a1) { z0 = (g11 * hb0 - g01 * hb1) / det; z1 = (g00 * hb1 - g01 * hb0) / det; }
        else if (a0) z0 = hb0 / g00;
        else if (a1) z1 = hb1 / g11;
        for (int c = 0; c < 3; ++c) {
            double vbar = W_src[c] * z0 + W_src[c + 3] * z1;
            double xc = x[c * n_px + i];
            int live = xc > 1.0 / 255.0 && xc < i0_in[c];
            grad_x[c * n_px + i] = live ? -vbar / xc : 0.0;
        }
    }
    memcpy(grad_W_tgt, dW, sizeof dW);
    free(H); free(mask); free(hbar);
    return flags;
}
