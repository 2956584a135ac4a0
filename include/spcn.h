/*
 * spcn.h -- C ABI of libspcn: structure-preserving color normalization (SPCN) on MI355X (gfx950).
 *
 * Method (arXiv 1901.03088, Sec. 2.1 and Sec. 3):
 *   Eq. (1)  optical density  v_c = log(i0_c / I_c) per channel and pixel;
 *   Eq. (2)  sparse NMF  min ||V - W H||_F^2 + lambda sum_j ||H(j,:)||_1 with W, H >= 0 and unit
 *            columns of W; with W fixed, H is found pixel by pixel (here: the exact non-negative
 *            lasso of each pixel, in closed form);
 *   Eq. (3)  V' = P99(H_tgt) / P99(H_src) * W_tgt H_src;
 *   Eq. (4)  I'_c = i0 exp(-V'_c);
 *   Sec. 3.1 item 2: the basis is fitted on sampled non-white pixels and the percentile is taken
 *   over non-white pixels only; Sec. 3.1 item 3: stains ordered by red-minus-blue OD.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller, unless marked "host".  The
 *     library never allocates or frees caller-visible memory.  Scratch memory comes from the
 *     caller's workspace `ws` (size from spcn_workspace_size); it needs no initialisation.
 *   - uint8 images are interleaved RGB (HWC), contiguous, 3 bytes per pixel, 4-byte aligned.
 *   - A stain basis W is 6 floats, 3x2 column-major: W[c + 3*j], c = R,G,B, j = 0 (hematoxylin),
 *     1 (eosin).  Entries must be non-negative (Eq. 2) and the columns non-parallel (unit norm is
 *     not required); any other basis is refused on the device (SPCN_FLAG_BASIS, densities 0).
 *   - Densities are planar FP32: H[j*n_px + i].
 *   - lambda follows Eq. (2) literally (no 1/2 on the squared error): a per-pixel penalty
 *     lambda*(h0 + h1) against ||v - W h||^2.
 *   - All work is enqueued on `stream`; nothing synchronises the host, allocates, or records a
 *     memset, so every entry point may be captured into a hipGraph.
 *   - Argument errors are detected on the host before anything is enqueued and returned as a
 *     status; spcn_last_error() then describes the problem (thread-local).  Conditions that depend
 *     on device data (no tissue, percentile in the overflow bin, degenerate basis) never abort:
 *     they are written as SPCN_FLAG_* bits into the caller's device `flags` words.
 *   - Nothing throws across this ABI and the library never prints.
 */
#ifndef SPCN_H
#define SPCN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPCN_OK = 0,
    SPCN_E_ARG = 1,          /* invalid argument: null pointer, size, range, alignment          */
    SPCN_E_WORKSPACE = 2,    /* workspace missing or smaller than spcn_workspace_size()         */
    SPCN_E_HIP = 3,          /* a HIP runtime call failed; spcn_last_error() has its message    */
    SPCN_E_UNSUPPORTED = 4   /* valid request this build does not implement                     */
} spcn_status;

/* Device-side result flags, one int32 word per stain (bit OR). */
#define SPCN_FLAG_NO_TISSUE 1   /* no pixel passed the non-white mask: scale kept at 1            */
#define SPCN_FLAG_RANGE     2   /* percentile fell in the last histogram bin (after the automatic
                                   retry, if any): raise hist_hi                                   */
#define SPCN_FLAG_BIN0      4   /* percentile fell in bin 0 (stain absent): scale kept at 1       */
#define SPCN_FLAG_BASIS     8   /* the basis is unusable (a negative or non-finite entry, or a
                                   singular Gram matrix): densities set to 0                        */
#define SPCN_FLAG_SHORT    16   /* basis estimation drew fewer tissue samples than requested      */
#define SPCN_FLAG_BATCH    32   /* batched call: this tile was skipped (bad descriptor, or total_px
                                   too small for the tiles)                                         */
#define SPCN_FLAG_TIMEOUT  64   /* a bounded device-side wait between workgroups expired: the
                                   results of this call are invalid                                 */
#define SPCN_FLAG_NO_BACKGROUND 128 /* spcn_estimate_i0 found no background pixel: i0 set to 255    */
#define SPCN_FLAG_RANGE_RETRY 256   /* the percentile fell in the last bin at the range given; the
                                       histogram was rebuilt at twice this stain's range (auto_range) */
#define SPCN_FLAG_SCALE    512  /* uint8 normalisation: the stain's scale_tgt is not finite and
                                   positive (NaN, infinite, zero or negative): scale kept at 1      */

#define SPCN_HIST_BINS 256

typedef struct {
    float i0[3];        /* Eq. (1) maximum intensity per channel (255 for 8-bit input; 1 for [0,1]) */
    float lambda;       /* Eq. (2) sparsity weight of the per-pixel density solve, >= 0            */
    int32_t white_sum;  /* non-white mask (Sec. 3.1 item 2): tissue iff R+G+B < white_sum; for float
                           input, iff 255*(x0+x1+x2) < white_sum in FP32; <= 0 disables the mask   */
    float percentile;   /* Eq. (3) percentile, in (0, 100]                                         */
    float hist_hi[2];   /* per-stain density histogram range [0, hist_hi): power of two in
                           [2^-8, 2^8]; 256 bins; values beyond land in the last bin               */
    const float* hist_hi_dev; /* device range that replaces hist_hi when non-NULL: [2] per image
                           ([n_tiles][2] for spcn_normalize_batched), e.g. the hist_hi_out of basis
                           estimation.  A value is rounded up to a power of two and clamped to
                           [2^-8, 2^8]; one that is not finite and positive falls back to hist_hi.
                           The histogram range is not part of the paper (Eq. 3 takes an order
                           statistic); it only places the bins.                                    */
    int32_t auto_range; /* 1: when a stain's percentile falls in the last bin, spcn_densities and
                           spcn_normalize rebuild the histogram once at twice that stain's range,
                           on the device (SPCN_FLAG_RANGE_RETRY); 0: only SPCN_FLAG_RANGE is set   */
} spcn_params;

/* Fills the paper's defaults: i0 = 255, lambda = 0.01, white_sum = 660 (mean intensity 220),
 * percentile 99, hist_hi = 4, no device range, auto_range = 1. */
void spcn_default_params(spcn_params* p);

/* Operation codes for spcn_workspace_size. */
#define SPCN_OP_DENSITIES         0   /* no size arguments */
#define SPCN_OP_NORMALIZE         1   /* no size arguments */
#define SPCN_OP_ESTIMATE_BASIS    2
#define SPCN_OP_NORMALIZE_BATCHED 3
#define SPCN_OP_ESTIMATE_BATCHED  4
#define SPCN_OP_FORWARD_F32       5
#define SPCN_OP_BACKWARD_F32      6
#define SPCN_OP_ESTIMATE_I0       7
#define SPCN_OP_SAMPLE_PERCENTILE 8   /* n_samples */
#define SPCN_OP_BAND_PERCENTILES  9   /* n_items = number of bands */
#define SPCN_OP_STREAM_NORMALIZE 10   /* n_px = image width, n_items = chunk_rows */
#define SPCN_OP_EXACT_PERCENTILE 11   /* no size arguments: a fixed 2^28 + 2^26 + 37120 bytes */
#define SPCN_OP_BANDWIDTH_PROBE  12   /* no size arguments: the read probe's 4 MiB sink */

/* Bytes of workspace the operation needs.  n_px: pixels per image (per sample for the float path);
 * n_items: images / tiles / samples; n_samples: pixels sampled for basis estimation.  Returns 0
 * for an unknown op. */
size_t spcn_workspace_size(int op, int64_t n_px, int64_t n_items, int64_t n_samples);

/* Densities of every pixel (Eq. 1 + Eq. 2 with W fixed) and their non-white histogram with its
 * percentile (Eq. 3 numerator when applied to a target image).
 *   img       uint8 HWC, height*width pixels
 *   w         [6] basis
 *   h_out     [2][n_px] FP32 densities, 16-byte aligned, or NULL (histogram only); each within
 *             2e-6 * max(1, hist_hi) of the exact value (fixed-point sums of 2^-16 bin when the
 *             basis allows them, else FP32 tables)
 *   hist_out  [2][256] uint64 counts over non-white pixels (overwritten)
 *   p99_out   [2] histogram percentile per stain (interpolated in the crossing bin), or NULL
 *   flags_out [2] SPCN_FLAG_* per stain, or NULL
 *   hist_hi_out [2] the range hist_out was built over (after an automatic retry), or NULL
 *   ws        spcn_workspace_size(SPCN_OP_DENSITIES, 0, 0, 0) bytes (range and retry words)
 * Histogram counts are exact: bin decisions agree with FP64 arithmetic on every pixel. */
spcn_status spcn_densities(const uint8_t* img, int64_t height, int64_t width, const float* w,
                           const spcn_params* p, float* h_out, uint64_t* hist_out, float* p99_out,
                           int32_t* flags_out, float* hist_hi_out, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/* Optional device outputs of spcn_normalize (any member may be NULL). */
typedef struct {
    uint64_t* hist;     /* [2][256] source histogram                    */
    float* p99_src;     /* [2] source percentile P99(H_src)             */
    float* scale;       /* [2] applied scale P99(H_tgt) / P99(H_src)    */
    int32_t* flags;     /* [2] SPCN_FLAG_* per stain                    */
    float* hist_hi;     /* [2] histogram range used (after an automatic retry) */
} spcn_norm_stats;

/* Fused normalisation of one uint8 image (Eqs. 1-4): pass 1 solves every pixel and builds the
 * non-white density histogram; pass 2 takes the percentile, scales, recolours with w_tgt and
 * writes uint8 (round half to even, clamped to [0, 255]).
 *   src, out   uint8 HWC images of height*width pixels (out may not alias src)
 *   w_src      [6] source basis;  w_tgt [6] target basis
 *   scale_tgt  [2] target percentiles P99(H_tgt) (e.g. p99_out of spcn_densities on the target);
 *              a stain whose value is not finite and positive is left unscaled (SPCN_FLAG_SCALE)
 *   i0_out     host [3] intensity of Eq. (4), or NULL for p->i0
 *   st         host struct of optional device outputs, or NULL
 *   ws         spcn_workspace_size(SPCN_OP_NORMALIZE, 0, 0, 0) bytes: histogram, range and retry
 *              words (the histogram goes to st->hist instead when that is given)
 * With p->auto_range, pass 1 is launched a second time; that launch ends at once unless a stain's
 * percentile fell in the last bin, in which case it rebuilds the histogram at twice that stain's
 * range (one retry, decided on the device, so the call stays free of host synchronisation). */
spcn_status spcn_normalize(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                           const float* w_tgt, const float* scale_tgt, const float* i0_out,
                           const spcn_params* p, uint8_t* out, const spcn_norm_stats* st,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/* spcn_normalize for callers that cannot allocate device memory (code under stream or graph
 * capture, serving loops, harnesses that forbid hipMalloc): the histogram and range words live in
 * a static device array of the library (8192 bytes per GPU, held until the process ends) instead
 * of a caller workspace.  The call itself allocates and frees nothing; the array's device address
 * is looked up once per device on the first call.  Arguments, results and errors as for
 * spcn_normalize (the needed scratch is fixed at 4352 bytes; a build needing more than the array
 * holds returns SPCN_E_WORKSPACE).  Every call on one GPU shares that GPU's array and leaves its
 * last contents there: the call clears what must start at zero, but two calls whose work overlaps
 * on one GPU (other streams, or host threads) race on it and must be serialised by the caller. */
spcn_status spcn_normalize_noalloc(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                                   const float* w_tgt, const float* scale_tgt, const float* i0_out,
                                   const spcn_params* p, uint8_t* out, const spcn_norm_stats* st,
                                   hipStream_t stream);

/* Pass 2 of spcn_normalize on its own: percentile of Eq. 3 from a given non-white histogram (from
 * spcn_densities on this image, or the element-wise sum of the histograms of its shards), scaling,
 * recolouring and Eq. 4.  Arguments as for spcn_normalize; hist is an input here and st->hist is
 * ignored.  The histogram's range is p->hist_hi_dev or p->hist_hi (no retry: the histogram is
 * given); st->hist_hi receives it.  spcn_densities followed by spcn_recolor (with hist_hi_dev =
 * the hist_hi_out of spcn_densities) equals spcn_normalize. */
spcn_status spcn_recolor(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                         const float* w_tgt, const float* scale_tgt, const float* i0_out,
                         const spcn_params* p, const uint64_t* hist, uint8_t* out,
                         const spcn_norm_stats* st, hipStream_t stream);

/* Out-of-core spcn_normalize for a slide in host memory (the paper's divide and conquer of WSIs,
 * Sec. 3.2 item 3, here for slides larger than, or arriving outside, device memory).  The slide is
 * processed in chunks of chunk_rows rows: pass 1 copies each chunk to the device and adds it to one
 * exact non-white histogram, pass 2 recolours it and copies the result back.  The first R chunks
 * stay resident in the workspace between the passes (R = spcn_stream_resident_chunks: as many as
 * the bytes beyond the minimum workspace hold); every other chunk is copied to the device again in
 * pass 2.  Copies run on copy_in / copy_out and overlap the kernels on `compute`; they start only
 * after the work queued on `compute` before the call; all work is enqueued without host
 * synchronisation and `compute` completes after the last copy.  The result equals spcn_normalize
 * of the whole slide byte for byte.
 *   host_src, host_out  uint8 HWC, 3*height*width bytes of pinned host memory (hipHostMalloc or
 *                       equivalent; pageable memory serialises the copies); they must not overlap
 *   chunk_rows          rows per chunk, at most 2^30 pixels per chunk
 *   st                  optional device statistics (hist is ignored: the histogram lives in ws)
 *   ws                  device workspace of at least spcn_workspace_size(SPCN_OP_STREAM_NORMALIZE,
 *                       width, chunk_rows, 0) bytes (the histogram and four chunk staging buffers);
 *                       each further 3*chunk_rows*width bytes (rounded up to 256) keep one more chunk
 *                       resident
 *   compute, copy_in, copy_out  streams; copy_in and copy_out must differ from compute (they may
 *                       be the same stream).  Overlapping calls on one device must be serialised. */
spcn_status spcn_normalize_streamed(const uint8_t* host_src, uint8_t* host_out, int64_t height,
                                    int64_t width, const float* w_src, const float* w_tgt,
                                    const float* scale_tgt, const float* i0_out,
                                    const spcn_params* p, int64_t chunk_rows,
                                    const spcn_norm_stats* st, void* ws, size_t ws_bytes,
                                    hipStream_t compute, hipStream_t copy_in, hipStream_t copy_out);

/* Number of chunks spcn_normalize_streamed keeps resident between its passes with a workspace of
 * ws_bytes bytes (0 for invalid sizes). */
int64_t spcn_stream_resident_chunks(int64_t height, int64_t width, int64_t chunk_rows, size_t ws_bytes);

/* Paper-compatible percentiles of Eq. 3 (alternatives to the exact global histogram percentile of
 * spcn_normalize; feed any of them to spcn_recolor_p99).
 *
 * spcn_band_percentiles: median of per-patch percentiles (Sec. 3.2 items 3-4: the slide processed
 * in longitudinal patches, the percentile taken as the median over patches).  Patches are bands of
 * band_rows full rows (the last one shorter); each band's percentile is the histogram percentile
 * of spcn_normalize over the band's non-white pixels (exact counts, p->hist_hi range); the median
 * over the bands holding non-white pixels is the middle value, or the mean of the two middle
 * values for an even count (0 and SPCN_FLAG_NO_TISSUE if none).
 *   band_rows  >= 1; at most 65536 bands
 *   band_p99   device [n_bands][2] per-band percentiles, or NULL;  p99_out device [2] medians
 *   flags_out  device [2] or NULL
 *   ws         spcn_workspace_size(SPCN_OP_BAND_PERCENTILES, 0, n_bands, 0) bytes */
spcn_status spcn_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                  const spcn_params* p, int64_t band_rows, float* band_p99,
                                  float* p99_out, int32_t* flags_out, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* spcn_sample_percentile: percentile of the sub-sampled non-white pixels (Sec. 3.1 item 2): the
 * densities (Eq. 2 with w fixed, p->lambda) of the first n_samples non-white pixels in the draw
 * order of spcn_estimate_basis (same seed, same draws), and per stain their nearest-rank
 * p->percentile: the k-th smallest with k = max(1, ceil(q n)).  Densities are computed in FP64.
 *   n_samples 1 .. 1048576;  p99_out device [2];  flags_out device [2] or NULL (SHORT, NO_TISSUE)
 *   ws        spcn_workspace_size(SPCN_OP_SAMPLE_PERCENTILE, 0, 0, n_samples) bytes */
spcn_status spcn_sample_percentile(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                   const spcn_params* p, int64_t n_samples, uint64_t seed,
                                   float* p99_out, int32_t* flags_out, void* ws, size_t ws_bytes,
                                   hipStream_t stream);

/* spcn_exact_percentile: the exact order statistic of Eq. 3 over all non-white pixels (Sec. 3.1
 * item 2), with no histogram interpolation: per stain the k-th smallest density (Eq. 2 with w fixed,
 * p->lambda, evaluated in FP64), k = max(1, ceil(q n)) over the n non-white pixels (nearest rank).
 * Two reads of the image: the exact histogram of spcn_densities (p->hist_hi only places the bins;
 * any range gives the same value) finds the bin that holds rank k; a second pass counts the colours
 * of the pixels in that bin, and a radix selection over the FP64 densities of those colours picks
 * the value.
 *   p99_out   device [2]: the selected FP64 density rounded to FP32 (0 without tissue)
 *   flags_out device [2] or NULL: SPCN_FLAG_NO_TISSUE, SPCN_FLAG_BASIS
 *   ws        spcn_workspace_size(SPCN_OP_EXACT_PERCENTILE, 0, 0, 0) bytes (about 320 MiB, whatever the
 *             image size); calls that share a workspace must not overlap */
spcn_status spcn_exact_percentile(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                  const spcn_params* p, float* p99_out, int32_t* flags_out, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/* Pass 2 of spcn_normalize with the source percentiles given (device [2], from any of the modes
 * above or from the caller): s_j = scale_tgt_j / p99_src_j, or 1 (SPCN_FLAG_BIN0) where p99_src_j is
 * not > 0 (SPCN_FLAG_SCALE where scale_tgt_j is not finite and positive).  Other arguments as for
 * spcn_normalize (out may not alias src).  scale_out [2] and
 * flags_out [2] (device) may be NULL.  No workspace. */
spcn_status spcn_recolor_p99(const uint8_t* src, int64_t height, int64_t width, const float* w_src,
                             const float* w_tgt, const float* scale_tgt, const float* i0_out,
                             const spcn_params* p, const float* p99_src, uint8_t* out,
                             float* scale_out, int32_t* flags_out, hipStream_t stream);

/* Basis estimation (Eq. 2 with both factors free; Sec. 3.1 items 2-3, Sec. 3.2 item 2): draws
 * n_samples non-white pixels with a counter-based SplitMix64 stream (candidate t -> pixel
 * floor(splitmix64(seed + (t+1)*0x9E3779B97F4A7C15) * n_px / 2^64), first n_samples non-white
 * candidates in draw order, at most 64*n_samples candidates), then n_iter alternating exact
 * H-steps and block-coordinate W-steps on the non-negative unit ball, normalises the columns and
 * puts hematoxylin (larger red-minus-blue OD) first.
 *   lambda_nmf   Eq. (2) sparsity weight for the fit (0.1 in the paper), finite and >= 0
 *   n_samples    1 .. 262144;  n_iter 0 .. 100000
 *   w_init       [6] initial basis, or NULL for the unit reference H&E vectors
 *                [0.65, 0.70, 0.29] and [0.07, 0.99, 0.11]
 *   w_out        [6] fitted basis;  sample_p99 [2] nearest-rank percentile (p->percentile) of the
 *                fitted densities of the samples, or NULL;  flags_out [2] or NULL
 *   hist_hi_out  [2] histogram range for the passes, or NULL: per stain the power of two
 *                2^ceil(log2(2 * sample_p99_j)), clamped to [2^-4, 2^6] (feed it to
 *                spcn_params.hist_hi_dev: the image percentile then lands in the middle of the bins
 *                unless it is more than twice the sample's) */
spcn_status spcn_estimate_basis(const uint8_t* img, int64_t height, int64_t width,
                                const spcn_params* p, float lambda_nmf, int64_t n_samples,
                                uint64_t seed, int32_t n_iter, const float* w_init, float* w_out,
                                float* sample_p99, float* hist_hi_out, int32_t* flags_out, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* Channel-wise background intensity i0 (Sec. 3.1 item 1: the fixed maximum intensity of Eqs. 1
 * and 4 replaced by a per-image, per-channel estimate).  Draws pixels with the same counter-based
 * SplitMix64 stream as spcn_estimate_basis and keeps the first n_samples whose mean intensity is
 * above 220 (R + G + B > white_sum, strict; at most 64*n_samples candidates), then takes per
 * channel the nearest-rank `percentile` (80 in the paper) of their values: the k-th smallest with
 * k = max(1, ceil(percentile/100 * n)).
 *   n_samples   1 .. 1048576 (the paper uses at most 100000)
 *   white_sum   1 .. 765 (660 = mean 220)
 *   percentile  (0, 100]
 *   i0_out      device [3] float, written with integer values; 255 if no background pixel is found
 *   flags_out   device [1] int32 or NULL: SPCN_FLAG_NO_BACKGROUND, SPCN_FLAG_SHORT
 *   ws          workspace of spcn_workspace_size(SPCN_OP_ESTIMATE_I0, 0, 0, n_samples) bytes
 * The estimate is fed back as spcn_params.i0 (source, Eq. 1) and i0_out (target's, Eq. 4). */
spcn_status spcn_estimate_i0(const uint8_t* img, int64_t height, int64_t width, int64_t n_samples,
                             uint64_t seed, int32_t white_sum, float percentile, float* i0_out,
                             int32_t* flags_out, void* ws, size_t ws_bytes, hipStream_t stream);

/* One tile of a batch (device-resident descriptor array). */
typedef struct {
    const uint8_t* src;   /* uint8 HWC tile, 4-byte aligned */
    uint8_t* out;         /* uint8 HWC output of the same size */
    int64_t height, width;
} spcn_tile;

/* Basis estimation for every tile of a batch (same algorithm as spcn_estimate_basis, one
 * workgroup per tile).  tiles: device array of n_tiles descriptors; w_out [n_tiles][6];
 * sample_p99 [n_tiles][2] or NULL; hist_hi_out [n_tiles][2] or NULL (as in spcn_estimate_basis,
 * per tile: feed it to spcn_params.hist_hi_dev of spcn_normalize_batched); flags_out [n_tiles][2]
 * or NULL.  Tile t uses seed + t.  A
 * descriptor with a NULL source or no pixels is not read: its basis is the initial one, its
 * percentiles 0 and its flags SPCN_FLAG_SHORT | SPCN_FLAG_NO_TISSUE. */
spcn_status spcn_estimate_basis_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t max_tile_px,
                                        const spcn_params* p, float lambda_nmf, int64_t n_samples,
                                        uint64_t seed, int32_t n_iter, const float* w_init,
                                        float* w_out, float* sample_p99, float* hist_hi_out,
                                        int32_t* flags_out, void* ws, size_t ws_bytes,
                                        hipStream_t stream);

/* Normalises every tile of a batch to one target (Eqs. 1-4, each tile with its own basis
 * w_src[t] and its own percentile) with a fixed sequence of launches and no host synchronisation
 * (the call can be captured into a graph): per-tile set-up, a work plan, a persistent pass 1 over
 * all tiles' items, a per-tile percentile check, the retry round (a second pass 1 over the items of
 * the tiles whose range was doubled, and their check), and one grid-stride pass 2 over all tiles.
 *   tiles    device array of n_tiles descriptors (1 <= n_tiles <= 8192), 4-byte aligned pointers
 *   total_px an upper bound of the tiles' total pixel count (sizes the workspace; if the tiles hold
 *            more, nothing is processed and every tile's flags get SPCN_FLAG_BATCH)
 *   w_src [n_tiles][6]; w_tgt [6]; scale_tgt [2] (as for spcn_normalize); i0_out host [3] or NULL;
 *   p99_out, scale_out [n_tiles][2] or NULL; flags_out [n_tiles][2] or NULL;
 *   hist_out [n_tiles][2][256] uint64 or NULL: each tile's non-white histogram (at its final range).
 * Tile t's histogram range is p->hist_hi_dev[2t .. 2t+1] when given, else p->hist_hi; with
 * p->auto_range a tile whose percentile lands in the last bin is counted again at twice that stain's
 * range (SPCN_FLAG_RANGE_RETRY), as spcn_normalize does.  Results are identical to calling
 * spcn_normalize on each tile with that range and the same auto_range. */
spcn_status spcn_normalize_batched(const spcn_tile* tiles, int32_t n_tiles, int64_t total_px,
                                   const float* w_src, const float* w_tgt, const float* scale_tgt,
                                   const float* i0_out, const spcn_params* p, float* p99_out,
                                   float* scale_out, int32_t* flags_out, uint64_t* hist_out, void* ws,
                                   size_t ws_bytes, hipStream_t stream);

/* Differentiable float path (extension: normalisation as a training-time augmentation layer).
 * x, y: [n][3][height][width] FP32 in [0, 1] (p->i0 is the input's i0, normally 1).  Per-sample
 * parameters are read at sample*stride (stride 0 broadcasts one value): w_src (stride in floats,
 * 6 per basis), w_tgt (6), scale_tgt (2; used as given: a differentiable parameter is not refused,
 * so a NaN propagates as in any layer).  The percentile is the EXACT nearest-rank order statistic
 * of each sample's non-white densities, k = max(1, ceil(q * n)); the selected pixel (smallest index
 * among equal values) is returned in sel_idx so the backward pass can route its gradient.
 *   i0_out   host [3] output intensity of Eq. (4), or NULL for p->i0
 *   p99_out [n][2], scale_out [n][2], sel_idx [n][2] (int64), flags_out [n][2]: saved state. */
spcn_status spcn_normalize_f32(const float* x, int64_t n, int64_t height, int64_t width,
                               const float* w_src, int64_t w_src_stride, const float* w_tgt,
                               int64_t w_tgt_stride, const float* scale_tgt, int64_t scale_stride,
                               const float* i0_out, const spcn_params* p, float* y, float* p99_out,
                               float* scale_out, int64_t* sel_idx, int32_t* flags_out, void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* Adjoint of spcn_normalize_f32 with w_src held fixed (the mask and the rank selection are
 * piecewise constant): given dL/dy, returns dL/dx, dL/dw_tgt and dL/dscale_tgt.  Per pixel the
 * density Jacobian comes from the active set's KKT system (h_F = G_FF^-1 (W_F^T v - lambda/2));
 * the percentile contributes through the density of the selected pixel sel_idx.
 *   p99, sel_idx, flags: the forward's saved outputs
 *   grad_x [n][3][h][w]
 *   grad_w_tgt  [n][6] per sample when w_tgt_stride > 0; [6] when the basis is shared by the batch
 *               (w_tgt_stride 0): the sum of the per-sample gradients, taken in sample order in FP64
 *   grad_scale  likewise: [n][2] when scale_stride > 0, else [2], the sum over samples. */
spcn_status spcn_normalize_backward(const float* x, int64_t n, int64_t height, int64_t width,
                                    const float* w_src, int64_t w_src_stride, const float* w_tgt,
                                    int64_t w_tgt_stride, const float* scale_tgt,
                                    int64_t scale_stride, const float* i0_out, const spcn_params* p,
                                    const float* p99, const int64_t* sel_idx, const int32_t* flags,
                                    const float* grad_y, float* grad_x, float* grad_w_tgt,
                                    float* grad_scale, void* ws, size_t ws_bytes,
                                    hipStream_t stream);

/* Memory-bandwidth reference for the roofline of the two passes (measurement only; it computes
 * nothing of the method): mode 0 copies `bytes` from src to dst (pass 2's traffic), mode 1 reads
 * them and XOR-reduces into the caller's workspace (pass 1's traffic), both grid-stride with
 * 16-byte accesses in the recolour pass's launch shape and with the passes' streaming cache policy
 * (non-temporal loads, non-temporal device-scope stores); modes 2 and 3 are the copy and the read
 * with the default cache policy.
 *   src, dst  device buffers, 16-byte aligned, not overlapping (dst unused in modes 1 and 3)
 *   bytes     a multiple of 16 in [16, 2^40]
 *   ws        modes 1, 3: spcn_workspace_size(SPCN_OP_BANDWIDTH_PROBE, 0, 0, 0) bytes; else unused */
spcn_status spcn_bandwidth_probe(const void* src, void* dst, int64_t bytes, int32_t mode, void* ws,
                                 size_t ws_bytes, hipStream_t stream);

/* Tuning options (autotuner hooks).  They select among kernel variants that compute identical
 * results; they are process-wide and read when work is enqueued.
 *   SPCN_OPT_P1_VARIANT        pass-1 table copies / histogram columns / units per thread and
 *                              iteration / workgroups per CU: 0 = (1, 64, 4, 1), 1 = (2, 64, 4, 1),
 *                              2 = (4, 32, 4, 1), 3 = (8, 16, 4, 1), 4 = (1, 32, 2, 2),
 *                              5 = (2, 16, 2, 2); 6, 7 = byte-permute table layout (8 copies,
 *                              16 columns), grid-stride tiles, 4 or 2 units per thread and
 *                              iteration; 8, 9 = narrow byte-permute layout (4 copies, 8 columns,
 *                              64 KB) with two 768- or 512-thread workgroups per CU (default 6)
 *   SPCN_OPT_P2_VARIANT        pass-2 table copies / workgroup size, contiguous chunks: 0 = (1, 256),
 *                              1 = (4, 256), 2 = (16, 1024); grid-stride tiles: 3 = (1, 256),
 *                              4 = (1, 512), 5 = (16, 1024) (default 3)
 *   SPCN_OPT_P2_BLOCKS_PER_CU  pass-2 workgroups per compute unit, 1..16 (default 8)
 *   SPCN_OPT_BATCH_CHUNK       batched normalisation: log2 of the 4-pixel units in one work item,
 *                              12..18 (default 15 = 131072 pixels)
 * spcn_set_option returns SPCN_E_ARG for an unknown option or a value out of range. */
#define SPCN_OPT_P1_VARIANT       0
#define SPCN_OPT_P2_VARIANT       1
#define SPCN_OPT_P2_BLOCKS_PER_CU 2
#define SPCN_OPT_BATCH_CHUNK      3
spcn_status spcn_set_option(int option, int value);
/* Current value of an option, or -1 for an unknown option. */
int spcn_get_option(int option);

/* Static description of a status code. */
const char* spcn_status_string(spcn_status s);
/* Detail of the last error returned on this thread ("" if none). */
const char* spcn_last_error(void);
/* Library version string. */
const char* spcn_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPCN_H */
