// spcn_basis.hip -- stain-basis estimation on gfx950: sample non-white pixels, fit the sparse NMF of
// Eq. (2) (Sec. 2.1 step 2), normalise the columns and put hematoxylin first (Sec. 3.1 item 3).
//
// Sampling (Sec. 3.1 item 2, Sec. 3.2 item 2): candidate t is pixel floor(z_t * n_px / 2^64) with
// z_t the SplitMix64 finaliser of seed + (t+1)*0x9E3779B97F4A7C15 (Steele, Lea & Flood 2014);
// the first n_s non-white candidates in draw order are kept, at most 64*n_s candidates are drawn.
//
// Fit: T rounds of (exact H-step for every sample with W fixed) then (one block-coordinate pass over
// the two columns of W, each the projection onto {w >= 0, ||w|| <= 1} of the column's unconstrained
// least-squares update u = w_j + (B_j - W A_j) / A_jj, with A = H H^T, B = V H^T).  The unit-norm
// equality of Eq. (2) is imposed after the last round.  The fit is small (<= a few 10^5 samples), so
// it runs in FP64 throughout (FP64 vector rate equals FP32 scalar rate on this chip); reductions
// have a fixed order, so results are bitwise reproducible (the exchanged partial sums lose their
// lowest mantissa bit to the round tag).
//
// Two layouts:
//   * one image with many samples: one launch for all rounds, up to 64 workgroups holding 4096
//     samples each in registers; per round FP64 partial sums per workgroup published as words
//     tagged with the round, and the same fixed-order reduction and W-step in every workgroup;
//   * a batch of tiles: one 256-thread workgroup per tile, samples held in registers, every round
//     inside the workgroup.
#include "spcn_internal.h"
#include "spcn_device.hpp"

namespace spcn {

namespace {

constexpr int SAMPLE_BLOCK = 1024;     // candidates per workgroup and round
constexpr int MAX_ROUNDS = 2;          // candidate budget 4 and 60 times n_s (the second round ends at once
                                       // when the first found enough: three small launches instead of six)
constexpr int TILE_THREADS = 256;
constexpr int TILE_SPT = 16;           // samples per thread in the batched kernel (n_s <= 4096)

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t candidate_pixel(uint64_t seed, uint64_t t, int64_t n_px) {
    return (int64_t)__umul64hi(splitmix64(seed, t), (uint64_t)n_px);
}

__device__ __forceinline__ bool non_white(const uint8_t* img, int64_t i, int32_t white_sum) {
    if (white_sum <= 0) return true;
    const uint8_t* p = img + 3 * i;
    return (int32_t)p[0] + (int32_t)p[1] + (int32_t)p[2] < white_sum;
}

// Block-wide exclusive prefix count of a predicate (blockDim.x multiple of 64).  Returns this
// thread's rank among the set predicates; *total receives the block's count.
__device__ int block_rank(bool pred, int* s_wave, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t m = __ballot(pred);
    const int below = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) s_wave[wave] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        int c = s_wave[w];
        off += (w < wave) ? c : 0;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return off + below;
}

// One DPP lane exchange of a double (both halves moved by the same control).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum of a double over the 64 lanes of a wavefront, in a fixed order, returned to every lane:
// butterflies inside each row of 16 lanes with DPP (quad xor 1, quad xor 2, half-row mirror, row
// mirror: each pairs two disjoint groups that already hold their partial sums), then the four row
// sums read from lanes 0, 16, 32, 48.  No LDS traffic.
__device__ __forceinline__ double wave_sum_d(double x) {
    x += dpp_d<0xB1>(x);     // quad_perm [1,0,3,2]
    x += dpp_d<0x4E>(x);     // quad_perm [2,3,0,1]
    x += dpp_d<0x141>(x);    // row_half_mirror
    x += dpp_d<0x140>(x);    // row_mirror
    const double r0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 0),
                                       __builtin_amdgcn_readlane(__double2loint(x), 0));
    const double r1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 16),
                                       __builtin_amdgcn_readlane(__double2loint(x), 16));
    const double r2 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 32),
                                       __builtin_amdgcn_readlane(__double2loint(x), 32));
    const double r3 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), 48),
                                       __builtin_amdgcn_readlane(__double2loint(x), 48));
    return (r0 + r1) + (r2 + r3);
}

// Sums of N values over the workgroup (wavefront DPP sums, then the waves in order); the totals
// land in out[0..N) (shared) for every thread.  Fixed association: deterministic.  Requires all
// lanes of every wavefront active.
template <int N>
__device__ inline void block_sums(double (&v)[N], double* s_red, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int q = 0; q < N; ++q) v[q] = wave_sum_d(v[q]);
    if (lane == 0)
        for (int q = 0; q < N; ++q) s_red[q * 16 + wave] = v[q];
    __syncthreads();
    if (threadIdx.x < N) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += s_red[threadIdx.x * 16 + w];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// FP64 basis for the H-step: Gram matrix and its determinant, from a double W.
struct NmfBasis {
    double w[6];
    double g00, g01, g11, det, half_lambda;
    double r_det, r00, r11;     // reciprocals of det, g00, g11 (the H-step multiplies)
    int ok;
};

__device__ inline void nmf_basis(const double* W, double lambda, NmfBasis& B) {
#pragma clang fp contract(off)
    for (int i = 0; i < 6; ++i) B.w[i] = W[i];
    double g00 = W[0] * W[0]; g00 = g00 + W[1] * W[1]; g00 = g00 + W[2] * W[2];
    double g01 = W[0] * W[3]; g01 = g01 + W[1] * W[4]; g01 = g01 + W[2] * W[5];
    double g11 = W[3] * W[3]; g11 = g11 + W[4] * W[4]; g11 = g11 + W[5] * W[5];
    B.g00 = g00; B.g01 = g01; B.g11 = g11;
    B.det = g00 * g11 - g01 * g01;
    B.half_lambda = 0.5 * lambda;
    B.ok = g00 > 0.0 && g11 > 0.0 && B.det > 0.0;
    B.r_det = B.ok ? 1.0 / B.det : 0.0;
    B.r00 = B.ok ? 1.0 / g00 : 0.0;
    B.r11 = B.ok ? 1.0 / g11 : 0.0;
}

// Exact non-negative lasso of one sample (Eq. 2 with W fixed): h_j = max(0, min(p_j, f_j)) with
// f = G^-1 b, p_j = b_j / g_jj (valid because g01 >= 0 for a non-negative W).  Columns of zero
// norm give zero densities.
__device__ __forceinline__ void nmf_rhs(const NmfBasis& B, double v0, double v1, double v2, double& b0, double& b1) {
    const double* W = B.w;
    b0 = W[0] * v0; b0 = b0 + W[1] * v1; b0 = b0 + W[2] * v2; b0 = b0 - B.half_lambda;
    b1 = W[3] * v0; b1 = b1 + W[4] * v1; b1 = b1 + W[5] * v2; b1 = b1 - B.half_lambda;
}

// The regular case (B.ok): branch-free.  SUMS: for the W-step's sums only, where the minimum may be
// the hardware one (v_min_f64, which may return -0 where the compare-select returns +0; a signed
// zero density adds the same zero to every sum).
template <bool SUMS = false>
__device__ __forceinline__ void nmf_solve_regular(const NmfBasis& B, double v0, double v1, double v2, double& h0,
                                                  double& h1) {
    double b0, b1;
    nmf_rhs(B, v0, v1, v2, b0, b1);
    double f0 = (B.g11 * b0 - B.g01 * b1) * B.r_det;
    double f1 = (B.g00 * b1 - B.g01 * b0) * B.r_det;
    double p0 = b0 * B.r00, p1 = b1 * B.r11;
    double t0, t1;
    if constexpr (SUMS) {
        t0 = __builtin_fmin(p0, f0);
        t1 = __builtin_fmin(p1, f1);
    } else {
        t0 = p0 < f0 ? p0 : f0;
        t1 = p1 < f1 ? p1 : f1;
    }
    h0 = t0 > 0.0 ? t0 : 0.0;
    h1 = t1 > 0.0 ? t1 : 0.0;
}

__device__ inline void nmf_solve(const NmfBasis& B, double v0, double v1, double v2, double& h0, double& h1) {
    if (B.ok) {
        nmf_solve_regular(B, v0, v1, v2, h0, h1);
    } else {
        double b0, b1;
        nmf_rhs(B, v0, v1, v2, b0, b1);
        double p0 = B.g00 > 0.0 ? b0 / B.g00 : 0.0, p1 = B.g11 > 0.0 ? b1 / B.g11 : 0.0;
        // one live column (or none): the problem is a scalar lasso in the better one
        double o0 = -p0 * b0, o1 = -p1 * b1;   // objective drop of each single-column candidate
        h0 = 0.0; h1 = 0.0;
        if (p0 > 0.0 && (o0 <= o1 || !(p1 > 0.0))) h0 = p0;
        else if (p1 > 0.0) h1 = p1;
    }
}

// The W-step's sums over one thread's samples (densities by the H-step above, then the products).
// Slots past the last sample hold v = 0, whose densities are exactly 0 (b = -lambda/2 <= 0 gives
// p <= 0), so they add exact zeros and need no test; with a regular basis (uniform over the
// workgroup) the loop is branch-free.
template <int K>
__device__ __forceinline__ void nmf_sums(const NmfBasis& B, const double (&v)[K][3], double (&acc)[9]) {
    auto add = [&](const double* x, double h0, double h1) {
        acc[0] += h0 * h0; acc[1] += h0 * h1; acc[2] += h1 * h1;
        acc[3] += x[0] * h0; acc[4] += x[0] * h1;
        acc[5] += x[1] * h0; acc[6] += x[1] * h1;
        acc[7] += x[2] * h0; acc[8] += x[2] * h1;
    };
    if (__builtin_amdgcn_readfirstlane(B.ok)) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double h0, h1;
            nmf_solve_regular<true>(B, v[k][0], v[k][1], v[k][2], h0, h1);
            add(v[k], h0, h1);
        }
    } else {
        for (int k = 0; k < K; ++k) {
            double h0, h1;
            nmf_solve(B, v[k][0], v[k][1], v[k][2], h0, h1);
            add(v[k], h0, h1);
        }
    }
}

// One block-coordinate pass of the W-step from the 9 sums (A00, A01, A11, B00, B01, B10, B11, B20,
// B21 with B_cj = sum v_c h_j), in place on W.
__device__ inline void w_step(double* W, const double* s) {
#pragma clang fp contract(off)
    const double A[2][2] = {{s[0], s[1]}, {s[1], s[2]}};
    for (int j = 0; j < 2; ++j) {
        if (!(A[j][j] > 0.0)) continue;                 // stain unused by every sample: keep w_j
        double u[3], nrm2 = 0.0;
        const double rA = 1.0 / A[j][j];
        for (int c = 0; c < 3; ++c) {
            double WAj = W[c] * A[0][j] + W[c + 3] * A[1][j];
            double Bcj = s[3 + 2 * c + j];
            double uc = W[c + 3 * j] + (Bcj - WAj) * rA;
            u[c] = uc > 0.0 ? uc : 0.0;
            nrm2 = nrm2 + u[c] * u[c];
        }
        if (!(nrm2 > 0.0)) continue;                    // projection is zero: keep w_j
        double sc = nrm2 > 1.0 ? 1.0 / sqrt(nrm2) : 1.0;
        for (int c = 0; c < 3; ++c) W[c + 3 * j] = u[c] * sc;
    }
}

// Unit columns, then hematoxylin (larger red-minus-blue OD) first.
__device__ inline void finish_basis(double* W) {
#pragma clang fp contract(off)
    for (int j = 0; j < 2; ++j) {
        double n = sqrt(W[3 * j] * W[3 * j] + W[3 * j + 1] * W[3 * j + 1] + W[3 * j + 2] * W[3 * j + 2]);
        if (n > 0.0)
            for (int c = 0; c < 3; ++c) W[c + 3 * j] /= n;
    }
    if (W[3] - W[5] > W[0] - W[2]) {
        for (int c = 0; c < 3; ++c) { double t = W[c]; W[c] = W[c + 3]; W[c + 3] = t; }
    }
}

__device__ inline void initial_basis(const float* w_init, double* W) {
    if (w_init) {
        for (int i = 0; i < 6; ++i) W[i] = (double)w_init[i];
        return;
    }
    // unit reference vectors of hematoxylin [0.65, 0.70, 0.29] and eosin [0.07, 0.99, 0.11], rounded
    // to FP32 like any basis handed to the library
    const double hr[3] = {0.65, 0.70, 0.29}, er[3] = {0.07, 0.99, 0.11};
    double nh = sqrt(hr[0] * hr[0] + hr[1] * hr[1] + hr[2] * hr[2]);
    double ne = sqrt(er[0] * er[0] + er[1] * er[1] + er[2] * er[2]);
    for (int c = 0; c < 3; ++c) {
        W[c] = (double)(float)(hr[c] / nh);
        W[c + 3] = (double)(float)(er[c] / ne);
    }
}

// The bin holding the kk-th smallest (1-based) value of a 256-bin digit histogram and kk's rank
// within that bin (s_misc[0], s_misc[1]), by a parallel inclusive scan: threads 0..255 one bin each
// (wavefront shuffles, then the four wavefront totals).  blockDim.x >= 256; ends with a barrier.
__device__ void pick_digit256(const uint32_t* s_hist, int64_t kk, uint32_t* s_wsum, int* s_misc) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint32_t c = 0, incl = 0;
    if (t < 256) {                      // whole wavefronts
        c = s_hist[t];
        incl = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        if (lane == 63) s_wsum[w] = incl;
    }
    if (t == 0) { s_misc[0] = 255; s_misc[1] = 1; }   // only if the counts fall short of kk
    __syncthreads();
    if (t < 256) {
        for (int i = 0; i < w; ++i) incl += s_wsum[i];
        if ((int64_t)(incl - c) < kk && kk <= (int64_t)incl) {   // exactly one bin
            s_misc[0] = t;
            s_misc[1] = (int)(kk - (int64_t)(incl - c));
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------ one image, many samples

struct BasisWork {          // layout of the caller's workspace (single image)
    int64_t n_s, max_cand;
    int32_t n_acc;          // samples kept so far
    int32_t base;           // sampling: samples kept before the current round
    int32_t flags;          // SPCN_FLAG_TIMEOUT if a wait between workgroups expired
    double W[6];
};

constexpr int FIT_THREADS = 512;
constexpr int FIT_SPT = 8;
constexpr int FIT_PER_BLOCK = FIT_THREADS * FIT_SPT;
constexpr int FIT_MAX_BLOCKS = 64;               // kMaxBasisSamples / FIT_PER_BLOCK (one wavefront)
constexpr uint32_t FIT_SPIN_LIMIT = 1u << 20;
static_assert(FIT_MAX_BLOCKS * FIT_PER_BLOCK >= kMaxBasisSamples, "fit grid must cover every sample");
static_assert(FIT_MAX_BLOCKS <= 64, "one partial row per lane of the reducing wavefront");
// Exchange slot of one workgroup and round parity: one 128-byte line whose first 9 words hold the
// workgroup's sums as FP64 bit patterns with the lowest mantissa bit replaced by the round's tag
// (bit 1 of the round number).  A slot of parity p is rewritten two rounds after it was read, so a
// word shows the tag of its round exactly when it holds that round's sum; the words start with tag 1
// (rounds 0 and 1 expect 0).  Readers clear the tag bit, so a sum reaches the W-step with its lowest
// mantissa bit cleared (within one unit in the last place; zero stays zero).
constexpr int FIT_SLOT = 16;                     // 64-bit words per slot: 9 tagged sums, padding
constexpr int FIT_SUMS = 9;
constexpr size_t FIT_XCHG_BYTES = (size_t)2 * FIT_MAX_BLOCKS * FIT_SLOT * sizeof(uint64_t);

__device__ __forceinline__ uint64_t* fit_slot(uint64_t* xchg, int parity, int b) {
    return xchg + ((size_t)parity * FIT_MAX_BLOCKS + b) * FIT_SLOT;
}
__device__ __forceinline__ uint64_t fit_tag(int round) { return (uint64_t)((round >> 1) & 1); }

struct SampleArgs {
    const uint8_t* img; int64_t n_px; int32_t white_sum; uint64_t seed;
    int32_t background;     // keep pixels with R + G + B > white_sum instead of non-white ones
    int64_t t0, t_end;      // candidates [t0, t_end) form this round
    int64_t nb;             // candidate groups in this round
    BasisWork* bw;
    uint64_t* staging;      // [nb][SAMPLE_BLOCK] kept candidates: pixel index | R << 40 | G << 48 | B << 56
    int32_t* counts;        // [nb + 1] kept candidates per group; the round's scan turns them into offsets
    int64_t* idx;           // [n_s] kept pixel indices
    const double* od;       // [3][256] optical densities (Eq. 1) when V is set
    double* V;              // [3][n_s] optical densities of the kept samples, or null
};

constexpr int STAGE_PIX_BITS = 40;   // pixel indices stay below 2^36 (the entry points' limit)

// Draws the round's candidate groups (SAMPLE_BLOCK candidates each, grid-stride, so that a round
// made unnecessary by earlier ones costs one small launch) and keeps each group's non-white
// candidates in draw order, with their bytes.
__global__ __launch_bounds__(SAMPLE_BLOCK) void k_sample_round(SampleArgs a) {
    __shared__ int s_wave[SAMPLE_BLOCK / 64];
    if (a.bw->n_acc >= a.bw->n_s) return;                  // earlier rounds found enough
    for (int64_t b = blockIdx.x; b < a.nb; b += gridDim.x) {
        const int64_t t = a.t0 + b * SAMPLE_BLOCK + threadIdx.x;
        bool keep = false;
        uint64_t packed = 0;
        if (t < a.t_end) {
            const int64_t pix = candidate_pixel(a.seed, (uint64_t)t, a.n_px);
            const uint8_t* q = a.img + 3 * pix;
            const uint32_t R = q[0], G = q[1], B = q[2];
            const int32_t sum = (int32_t)(R + G + B);
            keep = a.background ? sum > a.white_sum : (a.white_sum <= 0 || sum < a.white_sum);
            packed = (uint64_t)pix | ((uint64_t)R << STAGE_PIX_BITS) | ((uint64_t)G << (STAGE_PIX_BITS + 8)) |
                     ((uint64_t)B << (STAGE_PIX_BITS + 16));
        }
        int total;
        const int r = block_rank(keep, s_wave, &total);
        if (keep) a.staging[b * SAMPLE_BLOCK + r] = packed;
        if (threadIdx.x == 0) a.counts[b] = total;
    }
}

// Exclusive scan of the round's per-group counts (one workgroup), in place: counts[b] becomes the
// rank of group b's first kept candidate within the round and counts[nb] the round's total.
// Records the samples kept before the round and the new total (capped at n_s).
__global__ __launch_bounds__(1024) void k_sample_scan(SampleArgs a) {
    __shared__ int s_part[1024];
    BasisWork* bw = a.bw;
    const int t = threadIdx.x;
    if (bw->n_acc >= bw->n_s) {                 // earlier rounds found enough: nothing to append
        if (t == 0) bw->base = (int)bw->n_s;
        return;
    }
    const int nb = (int)a.nb;
    const int per = (nb + 1023) / 1024;
    int run = 0;
    for (int i = 0; i < per; ++i) {
        const int b = t * per + i;
        if (b < nb) run += a.counts[b];
    }
    s_part[t] = run;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = t >= o ? s_part[t - o] : 0;
        __syncthreads();
        s_part[t] += v;
        __syncthreads();
    }
    int off = t ? s_part[t - 1] : 0;
    for (int i = 0; i < per; ++i) {
        const int b = t * per + i;
        if (b < nb) {
            const int c = a.counts[b];
            a.counts[b] = off;
            off += c;
        }
    }
    if (t == 0) {
        const int base = bw->n_acc;
        a.counts[nb] = s_part[1023];
        bw->base = base;
        bw->n_acc = (int)min((int64_t)base + s_part[1023], bw->n_s);
    }
}

// Appends workgroup b's kept candidates of the round at their draw-order rank, while room is left.
__global__ __launch_bounds__(SAMPLE_BLOCK) void k_sample_copy(SampleArgs a) {
    const BasisWork* bw = a.bw;
    const int base = bw->base;
    const int64_t room = bw->n_s - base;
    if (room <= 0) return;
    for (int64_t b = blockIdx.x; b < a.nb; b += gridDim.x) {
        const int64_t off = a.counts[b];
        const int64_t c = a.counts[b + 1] - off;   // kept in this candidate group
        const int i = threadIdx.x;
        if (i < c && off + i < room) {
            const uint64_t packed = a.staging[b * SAMPLE_BLOCK + i];
            const int64_t k = base + off + i;
            a.idx[k] = (int64_t)(packed & ((1ull << STAGE_PIX_BITS) - 1));
            if (a.V) {
                const int64_t ns = bw->n_s;
                for (int ch = 0; ch < 3; ++ch)
                    a.V[ch * ns + k] = a.od[ch * kHistBins + (int)((packed >> (STAGE_PIX_BITS + 8 * ch)) & 255u)];
            }
        }
    }
}

// One sampling round: draw, scan, append (the three kernels above).
static void launch_round(const SampleArgs& a, const DevInfo& dev, hipStream_t s) {
    const int64_t cap = (int64_t)dev.cus * 4;
    const unsigned grid = (unsigned)(a.nb < cap ? a.nb : cap);
    hipLaunchKernelGGL(k_sample_round, dim3(grid), dim3(SAMPLE_BLOCK), 0, s, a);
    hipLaunchKernelGGL(k_sample_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_sample_copy, dim3(grid), dim3(SAMPLE_BLOCK), 0, s, a);
}

// Workspace state of a sampling run (one workgroup of 256 threads).  With od set, also the FP64
// optical densities od[c][k] of Eq. 1 for the given i0, which the copy stores per kept sample; with
// xchg set, the fit's exchange words start with a tag no round expects first.
__global__ __launch_bounds__(256) void k_basis_init(BasisWork* bw, int64_t n_s, int64_t max_cand, const float* w_init,
                                                    uint64_t* xchg, double* od, float i00, float i01, float i02) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        bw->n_s = n_s; bw->max_cand = max_cand; bw->n_acc = 0; bw->base = 0; bw->flags = 0;
        initial_basis(w_init, bw->W);
    }
    if (xchg)
        for (int i = threadIdx.x; i < 2 * FIT_MAX_BLOCKS * FIT_SUMS; i += blockDim.x)
            fit_slot(xchg, i / (FIT_MAX_BLOCKS * FIT_SUMS), (i / FIT_SUMS) % FIT_MAX_BLOCKS)[i % FIT_SUMS] = 1ull;
    if (od) {
        const float i0[3] = {i00, i01, i02};
        for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
            for (int c = 0; c < 3; ++c) od[c * kHistBins + k] = od_u8((double)i0[c], k);
    }
}

// The whole fit in one launch: every workgroup holds up to FIT_PER_BLOCK samples in registers for
// all rounds.  Per round each workgroup publishes its FP64 partial sums in its own slot (double-
// buffered by round parity) as tagged words (see fit_slot), each one relaxed 64-bit atomic store:
// the data is its own signal, so no release or acquire fence and no separate sequence word is
// needed.  One wavefront polls every workgroup's slot (a lane each) until all 9 words show the
// round's tag.  Then every workgroup reduces the same partials in the same fixed order and performs
// the same W-step, so all hold bit-identical W.  The grid (at most 64 workgroups) is far below what
// the chip keeps resident at once, so all workgroups run concurrently; the wait is bounded
// nonetheless and reports SPCN_FLAG_TIMEOUT.
struct FitArgs {
    BasisWork* bw;
    const double* V;        // [3][n_s]
    uint64_t* xchg;         // [2][FIT_MAX_BLOCKS][FIT_SLOT] tagged words, FIT_XCHG_BYTES
    double lambda;
    int32_t n_iter;
};

__global__ __launch_bounds__(FIT_THREADS) void k_nmf_fit(FitArgs a) {
    __shared__ double s_red[FIT_SUMS * 16];
    __shared__ NmfBasis s_B;         // the H-step constants of the current W
    __shared__ int s_abort;
    BasisWork* bw = a.bw;
    const int64_t n = bw->n_acc, ns = bw->n_s;
    const unsigned nblk = gridDim.x;
    double v[FIT_SPT][3];            // slots past the last sample hold zeros (they add nothing)
#pragma unroll
    for (int k = 0; k < FIT_SPT; ++k) {
        const int64_t i = (int64_t)blockIdx.x * FIT_PER_BLOCK + k * FIT_THREADS + threadIdx.x;
        for (int c = 0; c < 3; ++c) v[k][c] = i < n ? a.V[c * ns + i] : 0.0;
    }
    double W[6];                     // W in the registers of lane 0 (one W-step per workgroup and round)
    for (int i = 0; i < 6; ++i) W[i] = bw->W[i];
    if (threadIdx.x == 0) nmf_basis(W, a.lambda, s_B);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = FIT_THREADS >> 6;
    for (int it = 0; it < a.n_iter; ++it) {
        const NmfBasis B = s_B;
        double acc[FIT_SUMS] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        nmf_sums(B, v, acc);
        const int par = it & 1;
        const uint64_t tag = fit_tag(it);
        // the workgroup's sums (wavefront sums, then the waves in order), tagged, into its slot
        for (int q = 0; q < FIT_SUMS; ++q) acc[q] = wave_sum_d(acc[q]);
        if (lane == 0)
            for (int q = 0; q < FIT_SUMS; ++q) s_red[q * 16 + wave] = acc[q];
        __syncthreads();
        if (threadIdx.x < FIT_SUMS) {
            double t = 0.0;
            for (int w = 0; w < nw; ++w) t += s_red[threadIdx.x * 16 + w];
            const uint64_t word = ((uint64_t)__double_as_longlong(t) & ~1ull) | tag;
            __hip_atomic_store(fit_slot(a.xchg, par, blockIdx.x) + threadIdx.x, word, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x < 64) {  // one wavefront: lane b waits for workgroup b's words of this round
            bool ready = lane >= (int)nblk;
            uint64_t w[FIT_SUMS];
            for (int q = 0; q < FIT_SUMS; ++q) w[q] = 0ull;
            uint32_t spins = 0;
            int abort = 0;
            for (;;) {   // the slot's words and the abort flag are read together: one round trip per poll
                if (!ready) {
                    const uint64_t* src = fit_slot(a.xchg, par, lane);
                    uint64_t all = 1ull;
                    for (int q = 0; q < FIT_SUMS; ++q) {
                        w[q] = __hip_atomic_load(src + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        all &= ((w[q] & 1ull) == tag) ? 1ull : 0ull;
                    }
                    ready = all != 0ull;
                }
                const int stop = __hip_atomic_load(&bw->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                if (__ballot(!ready) == 0ull) break;
                if (++spins > FIT_SPIN_LIMIT || __builtin_amdgcn_readfirstlane(stop)) {
                    if (lane == 0) atomicOr(&bw->flags, SPCN_FLAG_TIMEOUT);
                    abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            double tot[FIT_SUMS];
            for (int q = 0; q < FIT_SUMS; ++q)
                tot[q] = (!abort && lane < (int)nblk) ? __longlong_as_double((long long)(w[q] & ~1ull)) : 0.0;
            for (int q = 0; q < FIT_SUMS; ++q) tot[q] = wave_sum_d(tot[q]);
            if (lane == 0) {       // every workgroup: the same update on the same sums
                s_abort = abort;
                if (!abort) {
                    w_step(W, tot);
                    nmf_basis(W, a.lambda, s_B);
                }
            }
        }
        __syncthreads();
        if (s_abort) return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int i = 0; i < 6; ++i) bw->W[i] = W[i];
}

// Unit columns, stain order, outputs and flags (one thread); the finished FP64 basis is kept in the
// workspace for the densities of the samples.
__global__ void k_nmf_finish(BasisWork* bw, float* w_out, int32_t* flags_out) {
    if (threadIdx.x != 0) return;
    double W[6];
    for (int i = 0; i < 6; ++i) W[i] = bw->W[i];
    finish_basis(W);
    for (int i = 0; i < 6; ++i) { bw->W[i] = W[i]; w_out[i] = (float)W[i]; }
    const int64_t n = bw->n_acc, ns = bw->n_s;
    if (flags_out)
        for (int j = 0; j < 2; ++j)
            flags_out[j] = (n < ns ? SPCN_FLAG_SHORT : 0) | (n == 0 ? SPCN_FLAG_NO_TISSUE : 0) | bw->flags;
}

// Fitted densities of the kept samples under the finished basis (the H-step of the fit, FP64),
// planar [2][n_s], for the sample percentile.
__global__ __launch_bounds__(256) void k_nmf_dens(const BasisWork* bw, const double* V, double lambda, double* H) {
    __shared__ NmfBasis s_B;
    if (threadIdx.x == 0) {
        double W[6];
        for (int i = 0; i < 6; ++i) W[i] = bw->W[i];
        nmf_basis(W, lambda, s_B);
    }
    __syncthreads();
    const NmfBasis B = s_B;
    const int64_t n = bw->n_acc, ns = bw->n_s;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double h0, h1;
        nmf_solve(B, V[i], V[ns + i], V[2 * ns + i], h0, h1);
        H[i] = h0;
        H[ns + i] = h1;
    }
}

// Nearest-rank percentile of each stain's sampled densities: a radix selection over the FP64 bit
// patterns (non-negative doubles order like them) spread over many workgroups.  Six digit passes of
// 11, 11, 11, 11, 11 and 8 bits (bit 63 is 0): k_sel_digits builds the digit histogram of the values
// that share the bits fixed so far, k_sel_pick fixes the next digit.
constexpr int SEL_BINS = 2048;
constexpr int SEL_PASSES = 6;
__host__ __device__ constexpr int sel_shift(int pass) { return pass < 5 ? 52 - 11 * pass : 0; }
__host__ __device__ constexpr int sel_width(int pass) { return pass < 5 ? 11 : 8; }

struct SelState {
    unsigned long long prefix[2];   // key bits fixed so far
    long long r[2];                 // 1-based rank still to find among the values sharing the prefix
    long long n;                    // values (kept samples)
    unsigned int n_cand[2];         // values gathered after the first two digits (may exceed SEL_CAND_CAP)
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// After two digits (22 key bits) few values still share the prefix: they are gathered once and the
// last four digits are taken over them inside one workgroup (over all values again if more than
// SEL_CAND_CAP share it, e.g. many equal densities).
constexpr int SEL_GATHER_PASSES = 2;
constexpr int SEL_CAND_CAP = 16384;

size_t sel_workspace_bytes() {
    return align256(sizeof(SelState)) + align256((size_t)2 * SEL_BINS * sizeof(uint32_t)) +
           align256((size_t)2 * SEL_CAND_CAP * sizeof(unsigned long long));
}

__global__ __launch_bounds__(64) void k_sel_init(const BasisWork* bw, double q, SelState* st, uint32_t* dhist) {
    const long long n = bw->n_acc;
    long long k = n > 0 ? (long long)ceil(q * (double)n) : 0;
    k = n > 0 ? (k < 1 ? 1 : (k > n ? n : k)) : 0;
    if (threadIdx.x < 2) { st->prefix[threadIdx.x] = 0ull; st->r[threadIdx.x] = k; st->n_cand[threadIdx.x] = 0u; }
    if (threadIdx.x == 0) st->n = n;
    for (int i = threadIdx.x; i < 2 * SEL_BINS; i += blockDim.x) dhist[i] = 0u;
}

__global__ __launch_bounds__(256) void k_sel_digits(const double* H, int64_t ns, const SelState* st, uint32_t* dhist,
                                                    int pass) {
    __shared__ uint32_t s_h[SEL_BINS];
    const int j = blockIdx.y;
    const long long n = st->n;
    if (n == 0) return;                                  // uniform
    for (int i = threadIdx.x; i < SEL_BINS; i += blockDim.x) s_h[i] = 0u;
    __syncthreads();
    const int shift = sel_shift(pass), hi = shift + sel_width(pass);
    const unsigned long long prefix = st->prefix[j], dmask = (1ull << sel_width(pass)) - 1;
    const double* Hj = H + j * ns;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double v = Hj[i];
        const unsigned long long u = v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
        if (((u ^ prefix) >> hi) == 0ull) atomicAdd(&s_h[(u >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SEL_BINS; i += blockDim.x)
        if (s_h[i]) atomicAdd(dhist + j * SEL_BINS + i, s_h[i]);
}

// Threads 0..255 of the workgroup: the bin of a 2048-bin digit histogram dh (global or LDS) that
// holds rank r (1-based, parallel prefix sums); returns the digit and the rank left inside its bin,
// valid in thread 0.  Barriers inside (every thread of the workgroup must call).
__device__ void sel_choose(const uint32_t* dh, uint32_t r, uint32_t* s_wsum, int* s_g, uint32_t* s_below,
                           uint32_t& digit, uint32_t& r_left) {
    const int t = threadIdx.x, lane = t & 63;
    constexpr int per = SEL_BINS / 256;
    uint32_t sum = 0, incl = 0;
    if (t < 256) {
#pragma unroll
        for (int i = 0; i < per; ++i) sum += dh[t * per + i];
        incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        if (lane == 63) s_wsum[t >> 6] = incl;
    }
    __syncthreads();
    if (t < 256) {
        for (int w = 0; w < (t >> 6); ++w) incl += s_wsum[w];
        if (t == 255) { *s_g = 255; *s_below = incl - sum; }   // default if the counts fall short of r
    }
    __syncthreads();
    if (t < 256 && incl - sum < r && r <= incl) { *s_g = t; *s_below = incl - sum; }   // at most one thread
    __syncthreads();
    if (t < 64) {
        const int g = *s_g;
        const uint32_t c = t < per ? dh[g * per + t] : 0u;
        uint32_t in = c;
        for (int o = 1; o < per; o <<= 1) {
            const uint32_t up = __shfl_up(in, o);
            if (t >= o) in += up;
        }
        const uint32_t rr = r - *s_below;
        const uint64_t m = __ballot(t < per && in - c < rr && rr <= in);
        const int who = m ? __ffsll((unsigned long long)m) - 1 : per - 1;
        const uint32_t before = __shfl(in - c, who);
        digit = (uint32_t)(g * per + who);
        r_left = rr - before;
    }
    __syncthreads();
}

// The value's outputs (thread 0 of the stain's workgroup).
__device__ void sel_outputs(const SelState* st, int j, int64_t ns, float* p99_out, int32_t* flags_out,
                            float* range_out) {
    const long long n = st->n;
    const double P = n > 0 ? __longlong_as_double((long long)st->prefix[j]) : 0.0;
    if (p99_out) p99_out[j] = (float)P;
    if (range_out) range_out[j] = range_for_percentile((double)(float)P);
    if (flags_out) flags_out[j] = (n == 0 ? SPCN_FLAG_NO_TISSUE : 0) | (n < ns ? SPCN_FLAG_SHORT : 0);
}

// One workgroup of 256 threads per stain: the digit holding the remaining rank, the digit histogram
// cleared for the next pass; after the last pass the value and the flags.
__global__ __launch_bounds__(256) void k_sel_pick(SelState* st, uint32_t* dhist, int pass, int64_t ns,
                                                  float* p99_out, int32_t* flags_out, float* range_out = nullptr) {
    __shared__ uint32_t s_wsum[4];
    __shared__ int s_g;
    __shared__ uint32_t s_below;
    const int j = blockIdx.x, t = threadIdx.x;
    const long long n = st->n;
    uint32_t* dh = dhist + j * SEL_BINS;
    if (n > 0) {
        uint32_t digit = 0, r_left = 0;
        sel_choose(dh, (uint32_t)st->r[j], s_wsum, &s_g, &s_below, digit, r_left);
        if (t == 0) {
            st->r[j] = (long long)r_left;
            st->prefix[j] |= (unsigned long long)digit << sel_shift(pass);
        }
        for (int i = t; i < SEL_BINS; i += blockDim.x) dh[i] = 0u;
    }
    if (pass == SEL_PASSES - 1 && t == 0) sel_outputs(st, j, ns, p99_out, flags_out, range_out);
}

// Gathers the key bits of the values that share the prefix of the first SEL_GATHER_PASSES digits
// (one append per wavefront: a ballot, one atomic, ranks by mbcnt).
__global__ __launch_bounds__(256) void k_sel_gather(const double* H, int64_t ns, SelState* st,
                                                    unsigned long long* cand) {
    const int j = blockIdx.y, lane = threadIdx.x & 63;
    const long long n = st->n;
    if (n == 0) return;                                  // uniform
    const int lo = sel_shift(SEL_GATHER_PASSES - 1);
    const unsigned long long prefix = st->prefix[j];
    const double* Hj = H + j * ns;
    unsigned long long* cj = cand + (int64_t)j * SEL_CAND_CAP;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i0 = (long long)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {   // uniform trip count
        const long long i = i0 + threadIdx.x;
        unsigned long long u = 0ull;
        bool keep = false;
        if (i < n) {
            const double v = Hj[i];
            u = v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
            keep = ((u ^ prefix) >> lo) == 0ull;
        }
        const uint64_t m = __ballot(keep);
        if (m == 0) continue;
        const int first = __ffsll((unsigned long long)m) - 1;
        uint32_t base = 0;
        if (lane == first) base = atomicAdd(&st->n_cand[j], (unsigned)__popcll(m));
        base = (uint32_t)__shfl((int)base, first);
        const uint32_t slot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (keep && slot < (uint32_t)SEL_CAND_CAP) cj[slot] = u;
    }
}

// The remaining digits in one workgroup of 256 threads per stain, over the gathered values (or over
// all values when more than SEL_CAND_CAP were gathered), then the outputs.
__global__ __launch_bounds__(256) void k_sel_finish(SelState* st, const unsigned long long* cand, const double* H,
                                                    int64_t ns, float* p99_out, int32_t* flags_out,
                                                    float* range_out) {
    __shared__ uint32_t s_h[SEL_BINS];
    __shared__ uint32_t s_wsum[4];
    __shared__ int s_g;
    __shared__ uint32_t s_below;
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_r;
    const int j = blockIdx.x, t = threadIdx.x;
    const long long n = st->n;
    if (n > 0) {
        const uint32_t c = st->n_cand[j];
        const bool gathered = c <= (uint32_t)SEL_CAND_CAP;
        const long long m = gathered ? (long long)c : n;
        const unsigned long long* cj = cand + (int64_t)j * SEL_CAND_CAP;
        const double* Hj = H + j * ns;
        if (t == 0) { s_prefix = st->prefix[j]; s_r = (uint32_t)st->r[j]; }
        for (int pass = SEL_GATHER_PASSES; pass < SEL_PASSES; ++pass) {
            for (int i = t; i < SEL_BINS; i += blockDim.x) s_h[i] = 0u;
            __syncthreads();
            const int shift = sel_shift(pass), hi = shift + sel_width(pass);
            const unsigned long long prefix = s_prefix, dmask = (1ull << sel_width(pass)) - 1;
            for (long long i = t; i < m; i += blockDim.x) {
                unsigned long long u;
                if (gathered) {
                    u = cj[i];
                } else {
                    const double v = Hj[i];
                    u = v > 0.0 ? (unsigned long long)__double_as_longlong(v) : 0ull;
                }
                if (((u ^ prefix) >> hi) == 0ull) atomicAdd(&s_h[(u >> shift) & dmask], 1u);
            }
            __syncthreads();
            uint32_t digit = 0, r_left = 0;
            sel_choose(s_h, s_r, s_wsum, &s_g, &s_below, digit, r_left);
            if (t == 0) { s_prefix |= (unsigned long long)digit << shift; s_r = r_left; }
            __syncthreads();
        }
        if (t == 0) { st->prefix[j] = s_prefix; st->r[j] = s_r; }
    }
    if (t == 0) sel_outputs(st, j, ns, p99_out, flags_out, range_out);
}

// ------------------------------------------------------------------ a batch of tiles

struct TileArgs {
    const spcn_tile* tiles;
    int32_t n_tiles;
    float i0[3];
    int32_t white_sum;
    double lambda;
    double q;
    int64_t n_s;
    uint64_t seed;
    int32_t n_iter;
    const float* w_init;
    float* w_out;
    float* sample_p99;
    float* range_out;
    int32_t* flags_out;
};

__global__ __launch_bounds__(TILE_THREADS) void k_nmf_tiles(TileArgs a) {
    __shared__ int64_t s_idx[TILE_THREADS * TILE_SPT];
    __shared__ double s_od[3 * kHistBins];
    __shared__ int s_wave[TILE_THREADS / 64];
    __shared__ double s_red[9 * 16];
    __shared__ double s_sum[9];
    __shared__ double s_W[6];
    __shared__ NmfBasis s_B;
    __shared__ uint32_t s_hist[256];
    __shared__ uint32_t s_wsum[4];
    __shared__ int s_misc[2];
    __shared__ int s_count;
    const int tile = blockIdx.x;
    const spcn_tile T = a.tiles[tile];
    // a descriptor without pixels (null source, zero or negative size) is never read: no samples
    const bool empty = T.src == nullptr || T.height <= 0 || T.width <= 0;
    const int64_t n_px = empty ? 0 : T.height * T.width;
    const uint64_t seed = a.seed + (uint64_t)tile;
    const int64_t n_s = a.n_s, max_cand = empty ? 0 : 64 * a.n_s;

    for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
        for (int c = 0; c < 3; ++c) s_od[c * kHistBins + k] = od_u8((double)a.i0[c], k);
    if (threadIdx.x == 0) { s_count = 0; initial_basis(a.w_init, s_W); }
    __syncthreads();

    // sampling, in draw order, one candidate per thread per step (four per thread and step, their
    // pixel reads unconditional and in flight together, measured 7% slower)
    for (int64_t t0 = 0; t0 < max_cand; t0 += blockDim.x) {
        const int base = s_count;
        if (base >= n_s) break;
        const int64_t t = t0 + threadIdx.x;
        bool keep = false;
        int64_t pix = 0;
        if (t < max_cand) {
            pix = candidate_pixel(seed, (uint64_t)t, n_px);
            keep = non_white(T.src, pix, a.white_sum);
        }
        int total;
        const int r = block_rank(keep, s_wave, &total);
        if (keep && base + r < n_s) s_idx[base + r] = pix;
        if (threadIdx.x == 0) s_count = (int)min((int64_t)base + total, n_s);
        __syncthreads();
    }
    const int n = s_count;

    // samples in registers: sample s lives in thread s % TILE_THREADS, slot s / TILE_THREADS
    double v[TILE_SPT][3];
    bool live[TILE_SPT];
#pragma unroll
    for (int k = 0; k < TILE_SPT; ++k) {
        const int s = k * TILE_THREADS + threadIdx.x;
        live[k] = s < n;
        const uint8_t* p = T.src + 3 * (live[k] ? s_idx[s] : 0);
        for (int c = 0; c < 3; ++c) v[k][c] = live[k] ? s_od[c * kHistBins + p[c]] : 0.0;
    }

    if (threadIdx.x == 0) nmf_basis(s_W, a.lambda, s_B);
    __syncthreads();
    for (int it = 0; it < a.n_iter; ++it) {
        const NmfBasis B = s_B;
        double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        nmf_sums(B, v, acc);
        block_sums(acc, s_red, s_sum);
        if (threadIdx.x == 0) {    // one W-step for the workgroup
            w_step(s_W, s_sum);
            nmf_basis(s_W, a.lambda, s_B);
        }
        __syncthreads();
    }
    double W[6];
    for (int i = 0; i < 6; ++i) W[i] = s_W[i];
    finish_basis(W);
    if (threadIdx.x == 0) {
        for (int i = 0; i < 6; ++i) a.w_out[6 * tile + i] = (float)W[i];
        if (a.flags_out)
            for (int j = 0; j < 2; ++j)
                a.flags_out[2 * tile + j] = (n < n_s ? SPCN_FLAG_SHORT : 0) | (n == 0 ? SPCN_FLAG_NO_TISSUE : 0);
    }
    if (!a.sample_p99 && !a.range_out) return;
    NmfBasis B;
    nmf_basis(W, a.lambda, B);
    double hv[TILE_SPT][2];
#pragma unroll
    for (int k = 0; k < TILE_SPT; ++k) nmf_solve(B, v[k][0], v[k][1], v[k][2], hv[k][0], hv[k][1]);
    for (int j = 0; j < 2; ++j) {
        double P = 0.0;
        if (n > 0) {
            int64_t kth = (int64_t)ceil(a.q * (double)n);
            kth = kth < 1 ? 1 : (kth > n ? n : kth);
            // radix select over the register-resident values: 8-bit digits of the FP64 bit patterns
            // (monotone for values >= 0) from the top, each digit picked by a parallel scan
            uint64_t prefix = 0, pmask = 0;
            int64_t kk = kth;
            for (int shift = 56; shift >= 0; shift -= 8) {
                for (int b = threadIdx.x; b < 256; b += blockDim.x) s_hist[b] = 0;
                __syncthreads();
#pragma unroll
                for (int k = 0; k < TILE_SPT; ++k) {
                    if (!live[k]) continue;
                    uint64_t u = (uint64_t)__double_as_longlong(hv[k][j]);
                    if ((u & pmask) == prefix) atomicAdd(&s_hist[(u >> shift) & 255], 1u);
                }
                __syncthreads();
                pick_digit256(s_hist, kk, s_wsum, s_misc);
                prefix |= (uint64_t)s_misc[0] << shift;
                pmask |= (uint64_t)255 << shift;
                kk = s_misc[1];
                __syncthreads();
            }
            P = __longlong_as_double((long long)prefix);
        }
        if (threadIdx.x == 0) {
            if (a.sample_p99) a.sample_p99[2 * tile + j] = (float)P;
            if (a.range_out) a.range_out[2 * tile + j] = range_for_percentile((double)(float)P);
        }
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

static int64_t hmin(int64_t a, int64_t b) { return a < b ? a : b; }

static int64_t round_candidates(int64_t n_s, int r) {
    const int64_t mult[MAX_ROUNDS] = {4, 60};
    return mult[r] * n_s;
}

static int64_t max_round_blocks(int64_t n_s) {
    return (round_candidates(n_s, MAX_ROUNDS - 1) + SAMPLE_BLOCK - 1) / SAMPLE_BLOCK;
}

size_t basis_workspace_bytes(int64_t n_s) {
    if (n_s <= 0) return 0;
    const int64_t nb = max_round_blocks(n_s);
    size_t b = align256(sizeof(BasisWork));
    b += align256((size_t)nb * SAMPLE_BLOCK * sizeof(uint64_t));  // staging
    b += align256((size_t)(nb + 1) * sizeof(int32_t));            // counts / offsets
    b += align256((size_t)n_s * sizeof(int64_t));                 // idx
    b += align256((size_t)3 * n_s * sizeof(double));              // V
    b += align256((size_t)3 * kHistBins * sizeof(double));        // optical-density table
    b += align256(FIT_XCHG_BYTES);                                // the fit's exchange slots
    b += align256((size_t)2 * n_s * sizeof(double));              // fitted densities of the samples
    b += sel_workspace_bytes();                                   // their percentile
    return b;
}

// Nearest-rank percentile of both stains of H [2][n_s] (the first bw->n_acc values of each row):
// the selection state, two digit passes over all values, the gathering of the values that share
// their prefix, the last digits in one workgroup per stain.  ws: sel_workspace_bytes().
static void launch_select(const BasisWork* bw, const double* H, int64_t n_s, double q, uint8_t* ws, float* p99_out,
                          int32_t* flags_out, const DevInfo& dev, hipStream_t s, float* range_out = nullptr) {
    SelState* sel = reinterpret_cast<SelState*>(ws);
    uint32_t* dhist = reinterpret_cast<uint32_t*>(ws + align256(sizeof(SelState)));
    unsigned long long* cand = reinterpret_cast<unsigned long long*>(
        ws + align256(sizeof(SelState)) + align256((size_t)2 * SEL_BINS * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(64), 0, s, bw, q, sel, dhist);
    const int64_t sel_want = hmin((n_s + 1023) / 1024, (int64_t)dev.cus);
    const unsigned sel_grid = (unsigned)(sel_want > 0 ? sel_want : 1);
    for (int pass = 0; pass < SEL_GATHER_PASSES; ++pass) {
        hipLaunchKernelGGL(k_sel_digits, dim3(sel_grid, 2), dim3(256), 0, s, H, n_s, (const SelState*)sel, dhist, pass);
        hipLaunchKernelGGL(k_sel_pick, dim3(2), dim3(256), 0, s, sel, dhist, pass, n_s, p99_out, flags_out, range_out);
    }
    hipLaunchKernelGGL(k_sel_gather, dim3(sel_grid, 2), dim3(256), 0, s, H, n_s, sel, cand);
    hipLaunchKernelGGL(k_sel_finish, dim3(2), dim3(256), 0, s, sel, (const unsigned long long*)cand, H, n_s, p99_out,
                       flags_out, range_out);
}

hipError_t launch_estimate_basis(const uint8_t* img, int64_t n_px, const ParamsK& pk, float lambda_nmf,
                                 int64_t n_s, uint64_t seed, int32_t n_iter, const float* w_init,
                                 float* w_out, float* sample_p99, float* range_out, int32_t* flags_out, void* ws,
                                 const DevInfo& dev, hipStream_t s) {
    const int nblk = (int)((n_s + FIT_PER_BLOCK - 1) / FIT_PER_BLOCK);
    if (nblk > FIT_MAX_BLOCKS) return hipErrorInvalidValue;
    uint8_t* p = static_cast<uint8_t*>(ws);
    BasisWork* bw = reinterpret_cast<BasisWork*>(p); p += align256(sizeof(BasisWork));
    const int64_t nbmax = max_round_blocks(n_s);
    uint64_t* staging = reinterpret_cast<uint64_t*>(p); p += align256((size_t)nbmax * SAMPLE_BLOCK * sizeof(uint64_t));
    int32_t* counts = reinterpret_cast<int32_t*>(p); p += align256((size_t)(nbmax + 1) * sizeof(int32_t));
    int64_t* idx = reinterpret_cast<int64_t*>(p); p += align256((size_t)n_s * sizeof(int64_t));
    double* V = reinterpret_cast<double*>(p); p += align256((size_t)3 * n_s * sizeof(double));
    double* od = reinterpret_cast<double*>(p); p += align256((size_t)3 * kHistBins * sizeof(double));
    uint64_t* xchg = reinterpret_cast<uint64_t*>(p); p += align256(FIT_XCHG_BYTES);
    double* H = reinterpret_cast<double*>(p); p += align256((size_t)2 * n_s * sizeof(double));
    uint8_t* sel_ws = p;

    const int64_t max_cand = 64 * n_s;
    hipLaunchKernelGGL(k_basis_init, dim3(1), dim3(256), 0, s, bw, n_s, max_cand, w_init, xchg, od, pk.i0[0], pk.i0[1],
                       pk.i0[2]);
    int64_t t0 = 0;
    for (int r = 0; r < MAX_ROUNDS && t0 < max_cand; ++r) {
        const int64_t rc = hmin(round_candidates(n_s, r), max_cand - t0);
        SampleArgs a{img, n_px, pk.white_sum, seed, 0, t0, t0 + rc, (rc + SAMPLE_BLOCK - 1) / SAMPLE_BLOCK, bw, staging,
                     counts, idx, od, V};
        launch_round(a, dev, s);
        t0 += rc;
    }
    FitArgs fa{bw, V, xchg, (double)lambda_nmf, n_iter};
    if (n_iter > 0) hipLaunchKernelGGL(k_nmf_fit, dim3(nblk), dim3(FIT_THREADS), 0, s, fa);
    hipLaunchKernelGGL(k_nmf_finish, dim3(1), dim3(64), 0, s, bw, w_out, flags_out);
    if (sample_p99 || range_out) {
        hipLaunchKernelGGL(k_nmf_dens, dim3((unsigned)hmin((n_s + 255) / 256, (int64_t)dev.cus * 4)), dim3(256), 0, s,
                           (const BasisWork*)bw, (const double*)V, (double)lambda_nmf, H);
        launch_select(bw, H, n_s, pk.q64, sel_ws, sample_p99, nullptr, dev, s, range_out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------- channel-wise background intensity

// Per-channel histogram of the sampled background pixels: workgroups take strided samples, count
// into per-wavefront LDS copies (background values crowd into a few bins) and add to the global
// [3][256] counts.
__global__ __launch_bounds__(1024) void k_i0_hist(const uint8_t* img, const int64_t* idx, const BasisWork* bw,
                                                  uint32_t* ghist) {
    __shared__ uint32_t s_hist[16][3 * kHistBins];
    const int t = threadIdx.x, wave = t >> 6;
    for (int i = t; i < 16 * 3 * kHistBins; i += blockDim.x) (&s_hist[0][0])[i] = 0u;
    __syncthreads();
    const int64_t n = bw->n_acc;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + t; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t* p = img + 3 * idx[i];
        atomicAdd(&s_hist[wave][p[0]], 1u);
        atomicAdd(&s_hist[wave][kHistBins + p[1]], 1u);
        atomicAdd(&s_hist[wave][2 * kHistBins + p[2]], 1u);
    }
    __syncthreads();
    for (int b = t; b < 3 * kHistBins; b += blockDim.x) {
        uint32_t sum = 0;
        for (int w = 0; w < 16; ++w) sum += s_hist[w][b];
        if (sum) atomicAdd(ghist + b, sum);
    }
}

__global__ void k_i0_clear(uint32_t* ghist) {
    for (int i = threadIdx.x; i < 3 * kHistBins; i += blockDim.x) ghist[i] = 0u;
}

// Nearest-rank percentile of each channel (one workgroup): k = max(1, ceil(q n)) in FP64, the
// smallest value whose cumulative count reaches k.
__global__ __launch_bounds__(256) void k_i0_select(const uint32_t* ghist, const BasisWork* bw, double q,
                                                   float* i0_out, int32_t* flags_out) {
    __shared__ uint32_t s_cum[3][kHistBins];
    const int t = threadIdx.x;
    if (t < 3) {   // 3 x 256 serial prefix sums
        uint32_t run = 0;
        for (int k = 0; k < kHistBins; ++k) { run += ghist[t * kHistBins + k]; s_cum[t][k] = run; }
    }
    __syncthreads();
    const int64_t n = bw->n_acc, ns = bw->n_s;
    if (n > 0) {
        int64_t k = (int64_t)ceil(q * (double)n);
        k = k < 1 ? 1 : (k > n ? n : k);
        for (int c = 0; c < 3; ++c)
            if ((int64_t)s_cum[c][t] >= k && (t == 0 || (int64_t)s_cum[c][t - 1] < k)) i0_out[c] = (float)t;
    } else if (t < 3) {
        i0_out[t] = 255.0f;
    }
    if (flags_out && t == 0)
        flags_out[0] = (n == 0 ? SPCN_FLAG_NO_BACKGROUND : 0) | (n < ns ? SPCN_FLAG_SHORT : 0);
}

size_t i0_workspace_bytes(int64_t n_s) {
    if (n_s <= 0) return 0;
    const int64_t nb = max_round_blocks(n_s);
    return align256(sizeof(BasisWork)) + align256((size_t)nb * SAMPLE_BLOCK * sizeof(uint64_t)) +
           align256((size_t)(nb + 1) * sizeof(int32_t)) + align256((size_t)n_s * sizeof(int64_t)) +
           align256((size_t)3 * kHistBins * sizeof(uint32_t));
}

hipError_t launch_estimate_i0(const uint8_t* img, int64_t n_px, int32_t white_sum, int64_t n_s, uint64_t seed,
                              double q, float* i0_out, int32_t* flags_out, void* ws, const DevInfo& dev,
                              hipStream_t s) {
    uint8_t* p = static_cast<uint8_t*>(ws);
    BasisWork* bw = reinterpret_cast<BasisWork*>(p); p += align256(sizeof(BasisWork));
    const int64_t nbmax = max_round_blocks(n_s);
    uint64_t* staging = reinterpret_cast<uint64_t*>(p); p += align256((size_t)nbmax * SAMPLE_BLOCK * sizeof(uint64_t));
    int32_t* counts = reinterpret_cast<int32_t*>(p); p += align256((size_t)(nbmax + 1) * sizeof(int32_t));
    int64_t* idx = reinterpret_cast<int64_t*>(p); p += align256((size_t)n_s * sizeof(int64_t));
    uint32_t* ghist = reinterpret_cast<uint32_t*>(p);
    const int64_t max_cand = 64 * n_s;
    hipLaunchKernelGGL(k_basis_init, dim3(1), dim3(256), 0, s, bw, n_s, max_cand, (const float*)nullptr,
                       (uint64_t*)nullptr, (double*)nullptr, 0.0f, 0.0f, 0.0f);
    hipLaunchKernelGGL(k_i0_clear, dim3(1), dim3(256), 0, s, ghist);
    int64_t t0 = 0;
    for (int r = 0; r < MAX_ROUNDS && t0 < max_cand; ++r) {
        const int64_t rc = hmin(round_candidates(n_s, r), max_cand - t0);
        SampleArgs a{img, n_px, white_sum, seed, 1, t0, t0 + rc, (rc + SAMPLE_BLOCK - 1) / SAMPLE_BLOCK, bw, staging,
                     counts, idx, nullptr, nullptr};
        launch_round(a, dev, s);
        t0 += rc;
    }
    hipLaunchKernelGGL(k_i0_hist, dim3((unsigned)hmin((n_s + 1023) / 1024, 128)), dim3(1024), 0, s, img,
                       (const int64_t*)idx, (const BasisWork*)bw, ghist);
    hipLaunchKernelGGL(k_i0_select, dim3(1), dim3(256), 0, s, (const uint32_t*)ghist, (const BasisWork*)bw, q,
                       i0_out, flags_out);
    return hipGetLastError();
}

// ------------------------------------------------- percentile of the sub-sampled pixels

// FP64 densities (Eq. 2, W fixed, the density lambda) of the sampled pixels, planar [2][n_s].
__global__ __launch_bounds__(256) void k_sample_dens(const uint8_t* img, const int64_t* idx, const BasisWork* bw,
                                                     const float* w, float lambda, float i00, float i01, float i02,
                                                     double* H) {
    __shared__ double s_od[3 * kHistBins];
    __shared__ Basis64 B;
    const float i0[3] = {i00, i01, i02};
    if (threadIdx.x == 0) derive_basis(w, lambda, B);
    for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
        for (int c = 0; c < 3; ++c) s_od[c * kHistBins + k] = od_u8((double)i0[c], k);
    __syncthreads();
    const int64_t n = bw->n_acc, ns = bw->n_s;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint8_t* p = img + 3 * idx[i];
        double h0 = 0.0, h1 = 0.0;
        if (B.ok) solve64(B, s_od[p[0]], s_od[kHistBins + p[1]], s_od[2 * kHistBins + p[2]], h0, h1);
        H[i] = h0;
        H[ns + i] = h1;
    }
}

size_t sample_pctl_workspace_bytes(int64_t n_s) {
    if (n_s <= 0) return 0;
    return i0_workspace_bytes(n_s) + align256((size_t)2 * n_s * sizeof(double)) + sel_workspace_bytes();
}

hipError_t launch_sample_percentile(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk, int64_t n_s,
                                    uint64_t seed, float* p99_out, int32_t* flags_out, void* ws, const DevInfo& dev,
                                    hipStream_t s) {
    uint8_t* p = static_cast<uint8_t*>(ws);
    BasisWork* bw = reinterpret_cast<BasisWork*>(p); p += align256(sizeof(BasisWork));
    const int64_t nbmax = max_round_blocks(n_s);
    uint64_t* staging = reinterpret_cast<uint64_t*>(p); p += align256((size_t)nbmax * SAMPLE_BLOCK * sizeof(uint64_t));
    int32_t* counts = reinterpret_cast<int32_t*>(p); p += align256((size_t)(nbmax + 1) * sizeof(int32_t));
    int64_t* idx = reinterpret_cast<int64_t*>(p); p += align256((size_t)n_s * sizeof(int64_t));
    double* H = reinterpret_cast<double*>(p); p += align256((size_t)2 * n_s * sizeof(double));
    uint8_t* sel_ws = p;
    const int64_t max_cand = 64 * n_s;
    hipLaunchKernelGGL(k_basis_init, dim3(1), dim3(256), 0, s, bw, n_s, max_cand, (const float*)nullptr,
                       (uint64_t*)nullptr, (double*)nullptr, 0.0f, 0.0f, 0.0f);
    int64_t t0 = 0;
    for (int r = 0; r < MAX_ROUNDS && t0 < max_cand; ++r) {
        const int64_t rc = hmin(round_candidates(n_s, r), max_cand - t0);
        SampleArgs a{img, n_px, pk.white_sum, seed, 0, t0, t0 + rc, (rc + SAMPLE_BLOCK - 1) / SAMPLE_BLOCK, bw, staging,
                     counts, idx, nullptr, nullptr};
        launch_round(a, dev, s);
        t0 += rc;
    }
    hipLaunchKernelGGL(k_sample_dens, dim3((unsigned)hmin((n_s + 255) / 256, (int64_t)dev.cus * 4)), dim3(256), 0, s,
                       img, (const int64_t*)idx, (const BasisWork*)bw, w, pk.lambda, pk.i0[0], pk.i0[1], pk.i0[2], H);
    launch_select(bw, H, n_s, pk.q64, sel_ws, p99_out, flags_out, dev, s);
    return hipGetLastError();
}

size_t basis_batched_workspace_bytes(int64_t, int64_t) { return 0; }

hipError_t launch_estimate_basis_batched(const spcn_tile* tiles, int32_t n_tiles, const ParamsK& pk,
                                         float lambda_nmf, int64_t n_s, uint64_t seed, int32_t n_iter,
                                         const float* w_init, float* w_out, float* sample_p99, float* range_out,
                                         int32_t* flags_out, void*, const DevInfo&, hipStream_t s) {
    TileArgs a{};
    a.tiles = tiles; a.n_tiles = n_tiles;
    for (int c = 0; c < 3; ++c) a.i0[c] = pk.i0[c];
    a.white_sum = pk.white_sum; a.lambda = (double)lambda_nmf; a.q = pk.q64; a.n_s = n_s; a.seed = seed;
    a.n_iter = n_iter; a.w_init = w_init; a.w_out = w_out; a.sample_p99 = sample_p99; a.range_out = range_out;
    a.flags_out = flags_out;
    hipLaunchKernelGGL(k_nmf_tiles, dim3(n_tiles), dim3(TILE_THREADS), 0, s, a);
    return hipGetLastError();
}

int64_t basis_tile_max_samples() { return (int64_t)TILE_THREADS * TILE_SPT; }

}  // namespace spcn
