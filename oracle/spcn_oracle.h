/*
 * spcn_oracle.h -- FP64 CPU oracle for structure-preserving color normalization (SPCN).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP library under paper_1901_03088_amd/)
 * never links, imports or calls it, and shares no source, header, table or constant with it.
 *
 * Everything here is plain, slow, FP64 arithmetic written straight from the paper's equations:
 *   Eq. (1)  optical density  v = log(i0 / i)                          (Sec. 2.1, step 1)
 *   Eq. (2)  sparse NMF  min ||V - W H||_F^2 + lambda * sum_j ||H(j,:)||_1,
 *            W >= 0, H >= 0, ||W(:,j)||_2^2 = 1                        (Sec. 2.1, step 2)
 *   Eq. (3)  V' = P99(H_tgt) / P99(H_src) * W_tgt H_src                (Sec. 2.1, step 3)
 *   Eq. (4)  i' = i0 exp(-v')                                           (Sec. 2.1, step 4)
 * plus the paper's fixes on this path: the non-white sample and the non-white percentile
 * (Sec. 3.1 item 2) and the red-minus-blue stain ordering (Sec. 3.1 item 3).
 *
 * Readings where the paper is silent are stated at each function.  Layouts: images are uint8 interleaved RGB (HWC), n_px pixels, 3*n_px bytes;
 * W is 3x2 column-major, W[c + 3*j] (c = R,G,B; j = stain 0 (hematoxylin), 1 (eosin));
 * densities are planar H[j*n + i].
 *
 * Parity status: every function below is pinned by the CPU tests in tests/test_oracle_*.py
 * (closed forms, brute force, library cross-checks, invariants).  No function is "parity unpinned".
 */
#ifndef SPCN_ORACLE_H
#define SPCN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes of the oracle's percentile / normalize steps (bit flags) */
#define ORC_OK         0
#define ORC_NO_TISSUE  1   /* no pixel passed the non-white mask: scale := 1                      */
#define ORC_RANGE      2   /* the percentile fell into the last (overflow) histogram bin           */
#define ORC_BIN0       4   /* the percentile fell into bin 0: the stain is absent, scale := 1      */
#define ORC_RANGE_RETRY 256 /* the range was doubled once because the percentile fell in the last bin */

/* Eq. (1) for one 8-bit channel; intensity 0 is read as 1 and OD is clamped at 0. */
double orc_od_u8(double i0, int intensity);
/* Eq. (1) for a float channel in [0,1] with i0 given; x is clamped below at 1/255. */
double orc_od_f(double i0, double x);

/* Eq. (2) with W fixed, one pixel: h = argmin_{h>=0} ||v - W h||^2 + lambda (h0 + h1), solved
 * by enumerating the four faces of the non-negative quadrant.  Returns the index of the winning
 * candidate (0: both zero, 1: only stain 0, 2: only stain 1, 3: both positive). */
int orc_solve_pixel(const double W[6], double lambda, const double v[3], double h[2]);

/* Non-white mask of Sec. 3.1 item 2: tissue iff R + G + B < white_sum (white_sum <= 0: all). */
int orc_is_tissue_u8(const uint8_t* px, int white_sum);

/* Densities of every pixel of a uint8 HWC image; H is planar [2][n_px]; mask (optional) gets 1 for tissue. */
void orc_densities_u8(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                      double lambda, int white_sum, double* H, uint8_t* mask);

/* 2 x bins histogram of tissue densities; bin width hist_hi[j] / bins; last bin takes the overflow. */
void orc_histogram(const double* H, const uint8_t* mask, int64_t n_px, const double hist_hi[2],
                   int bins, uint64_t* hist);

/* Percentile from one stain's histogram (interpolated inside the crossing bin).  Returns flags. */
int orc_percentile_hist(const uint64_t* counts, int bins, double hist_hi, double q, double* P, int* kstar);

/* Histogram range of each stain after the one automatic retry (the paper fixes no range for the
 * Eq. 3 percentile; the reading used: a stain whose percentile falls in the open last bin at
 * hist_hi[j] < 256 is counted again at 2 hist_hi[j], once).  range_out gets the settled ranges;
 * returns bit j set for each doubled stain. */
int orc_settle_range(const double* H, const uint8_t* mask, int64_t n_px, const double hist_hi[2], int bins,
                     double q, double range_out[2]);

/* Exact nearest-rank percentile of h over tissue pixels: the k-th smallest, k = max(1, ceil(q n)).
 * *idx = smallest linear index whose value equals the result.  Returns ORC_NO_TISSUE if n = 0. */
int orc_percentile_exact(const double* h, const uint8_t* mask, int64_t n_px, double q, double* P, int64_t* idx);

/* Full uint8 normalization (Eqs. 1-4) of one image, histogram percentile mode.
 * stats (optional, 8 doubles): P_src[2], scale[2], flags[2], n_tissue, unused.
 * hist_out (optional): the 2 x bins tissue histogram. */
int orc_normalize_u8(const uint8_t* src, int64_t n_px, const double W_src[6], const double W_tgt[6],
                     const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                     double lambda, int white_sum, double q, const double hist_hi[2], int bins,
                     uint8_t* out, double* stats, uint64_t* hist_out);

/* Eqs. (3)-(4) with the source percentiles given (any percentile mode below): the densities of
 * every pixel (Eq. 2 with W_src fixed), s_j = scale_tgt_j / P_src_j (1 where P_src_j is not > 0),
 * Eq. (4), round half to even, clamp.  out: 3*n_px bytes. */
void orc_recolor_u8(const uint8_t* src, int64_t n_px, const double W_src[6], const double W_tgt[6],
                    const double scale_tgt[2], const double P_src[2], const double i0_in[3],
                    const double i0_out[3], double lambda, int white_sum, uint8_t* out);

/* Median of per-patch percentiles (Sec. 3.2 items 3-4: the slide is processed in longitudinal
 * patches and the percentile of Eq. 3 is the median over patches of each patch's percentile).
 * Patches are bands of band_rows full rows (the last one shorter); each band's percentile is the
 * histogram percentile of orc_percentile_hist over its non-white pixels.  The median is taken over
 * the bands that hold non-white pixels: the middle value, or the mean of the two middle values
 * for an even count; with no such band it is 0 and ORC_NO_TISSUE is returned.  band_P and
 * band_flags (optional) receive [n_bands][2] values.  Returns the OR of the median's flags. */
int orc_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const double W[6],
                         const double i0[3], double lambda, int white_sum, double q,
                         const double hist_hi[2], int bins, int64_t band_rows, double* band_P,
                         int* band_flags, double median_P[2]);

/* Percentile of the sub-sampled non-white pixels (Sec. 3.1 item 2): the densities (Eq. 2, W fixed)
 * of the first n_s non-white pixels in the draw order of orc_sample_tissue, and per stain their
 * nearest-rank percentile q.  *kept receives the number of samples; with none, P = 0 and
 * ORC_NO_TISSUE is returned. */
int orc_sample_percentile(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                          double lambda, int white_sum, uint64_t seed, int64_t n_s, int64_t max_cand,
                          double q, double P[2], int64_t* kept);

/* Exact percentile of all non-white pixels (Eq. 3 over the pixels of Sec. 3.1 item 2, no histogram):
 * per stain the nearest-rank q order statistic of the FP64 densities (Eq. 2, W fixed) of the
 * non-white pixels.  *n_tissue receives their number; with none, P = 0 and ORC_NO_TISSUE is
 * returned. */
int orc_exact_percentile_u8(const uint8_t* img, int64_t n_px, const double W[6], const double i0[3],
                            double lambda, int white_sum, double q, double P[2], int64_t* n_tissue);

/* Per-pixel normalized intensity before rounding (used by the tests to locate rounding ties). */
void orc_reconstruct_pixel(const double h[2], const double W_tgt[6], const double s[2],
                           const double i0_out[3], double y[3]);

/* SplitMix64 finaliser (Steele, Lea & Flood 2014) applied to seed + (t+1) * golden gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t t);

/* Seeded sampling of non-white pixels (Sec. 3.1 item 2, Sec. 3.2 item 2): candidate t has index
 * floor(splitmix64(seed, t) * n_px / 2^64); tissue candidates are kept in order of t until n_s are
 * kept or max_cand candidates were drawn.  Returns the number kept. */
int64_t orc_sample_tissue(const uint8_t* img, int64_t n_px, int white_sum, uint64_t seed,
                          int64_t n_s, int64_t max_cand, int64_t* idx_out);

/* Channel-wise background intensity (Sec. 3.1 item 1: the fixed maximum intensity i0 of Eqs. (1)
 * and (4) replaced by a per-image, per-channel estimate).  Samples pixels whose mean intensity is
 * above 220 -- R + G + B > white_sum, strict, the complement of the non-white test without the
 * ties -- in the same SplitMix64 draw order as orc_sample_tissue (first n_s such candidates among at
 * most max_cand draws), and returns in i0_out[c] the nearest-rank percentile q (0.8 in the paper)
 * of channel c over the kept pixels: the k-th smallest value with k = max(1, ceil(q n)).  Returns
 * the number of pixels kept; with none kept, i0_out is left unchanged. */
int64_t orc_estimate_i0(const uint8_t* img, int64_t n_px, int white_sum, uint64_t seed, int64_t n_s,
                        int64_t max_cand, double q, double i0_out[3]);

/* Eq. (2) objective ||V - W H||_F^2 + lambda sum(H) over n columns, V is [3][n], H is [2][n]. */
double orc_nmf_objective(const double* V, const double* H, int64_t n, const double W[6], double lambda);

/* Sparse NMF by alternating exact H-steps and block-coordinate W-steps on the non-negative unit
 * ball, T iterations, then column normalisation and red-minus-blue ordering (Sec. 3.1 item 3).
 * V is [3][n] optical densities.  W_io: in = initial basis, out = fitted basis.  If obj_trace is
 * non-NULL it receives 2*T+1 objective values (before, after each H-step, after each W-step).
 * sample_p99 (optional) gets the exact nearest-rank 99th percentile of the final densities. */
void orc_nmf(const double* V, int64_t n, double lambda, int T, double W_io[6],
             double* obj_trace, double q, double* sample_p99);

/* Red-minus-blue stain order (Sec. 3.1 item 3): returns 1 if the columns must be swapped. */
int orc_stain_order_swap(const double W[6]);

/* Non-white mask for float pixels in [0,1]: the integer decision is taken in FP32, in this order:
 * s = (x0 + x1) + x2, tissue iff s * 255 < white_sum (white_sum <= 0: all pixels). */
int orc_is_tissue_f32(float x0, float x1, float x2, int white_sum);

/* Differentiable float path, one sample, CHW in [0,1] (plane stride n_px), i0 per channel.  x is
 * given in double so that finite differences can perturb it below FP32 resolution; the GPU input is
 * FP32 and is widened exactly.  The non-white mask rounds x to FP32 first (orc_is_tissue_f32).
 * Forward: exact-percentile scaling; saves P[2] and istar[2]; y is CHW. */
int orc_forward_f32(const double* x, int64_t n_px, const double W_src[6], const double W_tgt[6],
                    const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                    double lambda, int white_sum, double q, double* y, double* P, int64_t* istar,
                    double* H_out);

/* Per pixel of a float image (CHW), the distance from a change of the Eq. (2) active set:
 * min over |b_j / g_jj| and |(G^-1 b)_j| (if G is regular), b = W^T v - lambda/2. */
void orc_active_margin_f32(const double* x, int64_t n_px, const double W[6], const double i0_in[3],
                           double lambda, double* margin);

/* Analytic adjoint of orc_forward_f32 w.r.t. x, W_tgt and scale_tgt (W_src held fixed; the mask
 * and the rank selection are piecewise constant).  If istar_in is non-NULL it fixes the selected
 * pixels (else they are recomputed).  grad_x is CHW like x. */
int orc_backward_f32(const double* x, int64_t n_px, const double W_src[6], const double W_tgt[6],
                     const double scale_tgt[2], const double i0_in[3], const double i0_out[3],
                     double lambda, int white_sum, double q, const double* grad_y,
                     const int64_t* istar_in, double* grad_x, double grad_W_tgt[6],
                     double grad_scale[2]);

#ifdef __cplusplus
}
#endif
#endif
