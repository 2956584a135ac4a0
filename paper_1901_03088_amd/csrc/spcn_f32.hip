// spcn_f32.hip -- differentiable SPCN on float images (extension: normalisation as a training-time
// augmentation layer).  x, y: [n][3][H][W] FP32 in [0, 1]; per-sample source basis, target basis and
// target scales.  The percentile of Eq. 3 is the EXACT nearest-rank order statistic of each sample's
// non-white densities, so that its gradient can be routed to the selected pixel.
//
// Forward
//   k_fw_dens     densities of every pixel (Eq. 1 via v_log_f32, Eq. 2 closed form), stored with the
//                 sign bit marking white pixels; per-sample coarse histogram (2048 bins of width 1/256
//                 over [0, 8), last bin open) of the non-white densities, and the non-white count;
//   k_fw_bin      per (sample, stain): the coarse bin holding rank k = max(1, ceil(q n)) and the rank
//                 inside it;
//   k_fw_collect  appends (value, index) of every non-white pixel in that bin to a candidate list;
//   k_fw_select   per (sample, stain): radix selection of the rank among the candidates' values, then
//                 the smallest index holding that value; if the list overflowed, the same selection
//                 over the whole sample; writes P, the selected index, scale and recolouring constants;
//   k_fw_recon    Eqs. 3-4 from the stored densities.
// Backward (W_src fixed; the mask and the rank selection are piecewise constant)
//   k_bw_main     per pixel: ubar_c = -y_c gbar_c; hbar_j = s_j sum_c Wt[c,j] ubar_c; on the active set F
//                 of the pixel's KKT system vbar = W_F G_FF^-1 hbar_F; xbar_c = -vbar_c / x_c where the
//                 OD is not clamped; partial sums of dWt and ds (FP32 over a thread's few pixels, FP64
//                 across threads and workgroups);
//   k_bw_reduce   per sample: ordered sums -> dWt, dS = ds / P; the percentile's adjoint
//                 Pbar_j = -(s_j / P_j) ds_j enters through the selected pixel's density (added to
//                 its input gradient);
//   k_bw_shared   a target basis or scale shared by the batch: the sum over samples.
#include "spcn_internal.h"
#include "spcn_device.hpp"

#include <cmath>

namespace spcn {

namespace {

constexpr int FT = 256;               // threads per workgroup
constexpr int NBIN = 2048;            // coarse bins per stain
constexpr float BIN_SCALE = 256.0f;   // bins per density unit
constexpr int CAP = 16384;            // candidate capacity per (sample, stain)
constexpr int BLOCKS_PER_SAMPLE_MAX = 128;

struct F32Basis {          // FP32 constants of one sample's solve and recolouring
    float q[2][3];         // G^-1 W^T
    float fc[2];           // -lambda/2 G^-1 1
    float a[2];            // g01/g00, g01/g11
    float w[6];            // source basis (backward)
    float g00, g01, g11, det;
    float r_det, r00, r11;  // reciprocals of det, g00, g11 (0 for a singular basis)
    float i0[3], log2i0[3];
    int ok;
};

__device__ inline void f32_basis(const float* w, float lambda, const float i0[3], const float log2i0[3], F32Basis& F) {
    Basis64 B;
    derive_basis(w, lambda, B);
    for (int j = 0; j < 2; ++j) {
        for (int c = 0; c < 3; ++c) F.q[j][c] = (float)B.q[j][c];
        F.fc[j] = (float)B.fconst[j];
        F.a[j] = (float)B.a[j];
    }
    for (int i = 0; i < 6; ++i) F.w[i] = w[i];
    F.g00 = (float)B.g00; F.g01 = (float)B.g01; F.g11 = (float)B.g11; F.det = (float)B.det;
    F.r_det = B.ok ? (float)(1.0 / B.det) : 0.0f;
    F.r00 = B.g00 > 0.0 ? (float)(1.0 / B.g00) : 0.0f;
    F.r11 = B.g11 > 0.0 ? (float)(1.0 / B.g11) : 0.0f;
    for (int c = 0; c < 3; ++c) { F.i0[c] = i0[c]; F.log2i0[c] = log2i0[c]; }
    F.ok = B.ok;
}

struct Px {
    float od[3];
    bool live[3];          // OD neither clamped at 1/255 nor at 0 (derivative -1/x exists)
    float h0, h1;
    bool tissue;
};

// Eq. 1 + Eq. 2 of one float pixel, FP32.
__device__ __forceinline__ void solve_px(const F32Basis& F, float x0, float x1, float x2, int white_sum, Px& p) {
    const float xs[3] = {x0, x1, x2};
    const float lo = 1.0f / 255.0f;
    for (int c = 0; c < 3; ++c) {
        const float xc = fmaxf(xs[c], lo);
        const float v = (F.log2i0[c] - __builtin_amdgcn_logf(xc)) * 0.69314718055994531f;
        p.od[c] = fmaxf(v, 0.0f);
        // the clamp's kink is at the real 1/255, which lies just below its FP32 rounding lo: every
        // x >= lo is above the kink and has the derivative -1/x
        p.live[c] = xs[c] >= lo && xs[c] < F.i0[c];
    }
    float f0 = F.fc[0], f1 = F.fc[1];
    for (int c = 0; c < 3; ++c) { f0 = fmaf(F.q[0][c], p.od[c], f0); f1 = fmaf(F.q[1][c], p.od[c], f1); }
    p.h0 = F.ok ? fmaxf(0.0f, fmaf(F.a[0], fminf(f1, 0.0f), f0)) : 0.0f;
    p.h1 = F.ok ? fmaxf(0.0f, fmaf(F.a[1], fminf(f0, 0.0f), f1)) : 0.0f;
    if (white_sum <= 0) {
        p.tissue = true;
    } else {
        const float s = __fadd_rn(__fadd_rn(x0, x1), x2);
        p.tissue = __fmul_rn(s, 255.0f) < (float)white_sum;
    }
}

__device__ __forceinline__ int coarse_bin(float h) {
    const float b = h * BIN_SCALE;
    return b >= (float)(NBIN - 1) ? NBIN - 1 : (int)b;
}

struct SampleState {       // per sample, in the workspace
    uint32_t n_tissue;
    int32_t bin[2];        // coarse bin of the selected rank
    int32_t rank_in_bin[2];
    uint32_t n_cand[2];
    float P[2], s[2];
    int64_t sel[2];
    int32_t flags[2];
    float M[3][2], L[3];   // recolouring constants (log2 domain)
};

struct FwArgs {
    const float* x; int64_t n, n_px;
    const float* w_src; int64_t w_src_stride;
    const float* w_tgt; int64_t w_tgt_stride;
    const float* scale_tgt; int64_t scale_stride;
    float i0[3], i0_out[3], lambda;
    float log2i0[3], log2io[3];   // log2 of i0 and i0_out (host-computed)
    int32_t white_sum;
    double q;
    float* hstore;           // [n][2][n_px]
    uint32_t* chist;         // [n][2][NBIN]
    SampleState* st;         // [n]
    uint64_t* cand;          // [n][2][CAP] (value bits << 32 | index)
    float* y;
    float* p99_out; float* scale_out; int64_t* sel_idx; int32_t* flags_out;
};

__global__ void k_fw_clear(FwArgs a) {
    const int64_t total = a.n * 2 * NBIN;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
        a.chist[i] = 0u;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < a.n; s += (int64_t)gridDim.x * blockDim.x) {
        a.st[s].n_tissue = 0;
        a.st[s].n_cand[0] = 0; a.st[s].n_cand[1] = 0;
    }
}

// V pixels per thread and iteration: 4 when every plane is 16-byte aligned (n_px % 4 == 0 and aligned
// base pointers; one 16-byte access per plane), else 1.  The planes are streamed (each kernel reads
// and writes them once, and the batch does not stay cached between kernels): with NT the accesses
// are non-temporal, which measured faster in every kernel but the recolouring one.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int V, bool NT = true>
struct Vec;
template <bool NT>
struct Vec<1, NT> {
    static __device__ __forceinline__ void load(const float* p, float (&v)[1]) {
        v[0] = NT ? __builtin_nontemporal_load(p) : *p;
    }
    static __device__ __forceinline__ void store(float* p, const float (&v)[1]) {
        if (NT) __builtin_nontemporal_store(v[0], p);
        else *p = v[0];
    }
};
template <bool NT>
struct Vec<4, NT> {
    static __device__ __forceinline__ void load(const float* p, float (&v)[4]) {
        const f32x4* q = reinterpret_cast<const f32x4*>(p);
        const f32x4 t = NT ? __builtin_nontemporal_load(q) : *q;
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
    static __device__ __forceinline__ void store(float* p, const float (&v)[4]) {
        f32x4 t;
        t.x = v[0]; t.y = v[1]; t.z = v[2]; t.w = v[3];
        if (NT) __builtin_nontemporal_store(t, reinterpret_cast<f32x4*>(p));
        else *reinterpret_cast<f32x4*>(p) = t;
    }
};

template <int V>
__global__ __launch_bounds__(FT) void k_fw_dens(FwArgs a) {
    __shared__ uint32_t s_hist[2 * NBIN];
    __shared__ F32Basis F;
    __shared__ uint32_t s_count;
    const int64_t s = blockIdx.y;
    for (int i = threadIdx.x; i < 2 * NBIN; i += FT) s_hist[i] = 0u;
    if (threadIdx.x == 0) {
        f32_basis(a.w_src + s * a.w_src_stride, a.lambda, a.i0, a.log2i0, F);
        s_count = 0;
    }
    __syncthreads();
    const float* x = a.x + s * 3 * a.n_px;
    float* hs = a.hstore + s * 2 * a.n_px;
    uint32_t cnt = 0;
    const int64_t nq = a.n_px / V;
    for (int64_t q = blockIdx.x * (int64_t)FT + threadIdx.x; q < nq; q += (int64_t)gridDim.x * FT) {
        const int64_t i = q * V;
        float x0[V], x1[V], x2[V], h0[V], h1[V];
        Vec<V>::load(x + i, x0);
        Vec<V>::load(x + a.n_px + i, x1);
        Vec<V>::load(x + 2 * a.n_px + i, x2);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            Px p;
            solve_px(F, x0[k], x1[k], x2[k], a.white_sum, p);
            h0[k] = p.tissue ? p.h0 : -p.h0;
            h1[k] = p.tissue ? p.h1 : -p.h1;
            if (p.tissue) {
                ++cnt;
                atomicAdd(&s_hist[coarse_bin(p.h0)], 1u);
                atomicAdd(&s_hist[NBIN + coarse_bin(p.h1)], 1u);
            }
        }
        Vec<V>::store(hs + i, h0);
        Vec<V>::store(hs + a.n_px + i, h1);
    }
    atomicAdd(&s_count, cnt);
    __syncthreads();
    uint32_t* gh = a.chist + s * 2 * NBIN;
    for (int i = threadIdx.x; i < 2 * NBIN; i += FT)
        if (s_hist[i]) atomicAdd(gh + i, s_hist[i]);
    if (threadIdx.x == 0) atomicAdd(&a.st[s].n_tissue, s_count);
}

// rank k of the nearest-rank percentile among n values
__device__ inline int64_t pct_rank(double q, int64_t n) {
    int64_t k = (int64_t)ceil(q * (double)n);
    return k < 1 ? 1 : (k > n ? n : k);
}

// Inclusive prefix sum of one value per thread over the first 256 threads of the workgroup (wave
// scans, then the totals of the preceding waves); s_wsum holds 4 words.  Barriers inside.
__device__ inline uint32_t scan256(uint32_t v, uint32_t* s_wsum) {
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t up = __shfl_up(incl, o);
        if (lane >= o) incl += up;
    }
    if (tid < 256 && lane == 63) s_wsum[tid >> 6] = incl;
    __syncthreads();
    if (tid < 256)
        for (int w = 0; w < (tid >> 6); ++w) incl += s_wsum[w];
    __syncthreads();
    return incl;
}

__global__ __launch_bounds__(FT) void k_fw_bin(FwArgs a) {
    __shared__ uint32_t s_wsum[4];
    __shared__ int s_g;
    __shared__ uint32_t s_below;
    const int64_t s = blockIdx.x >> 1;
    const int j = blockIdx.x & 1;
    const int tid = threadIdx.x;
    const uint32_t* h = a.chist + (s * 2 + j) * NBIN;
    constexpr int per = NBIN / FT;             // bins per thread (FT == 256)
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) sum += h[tid * per + i];
    const int64_t n = a.st[s].n_tissue;
    const int64_t k = n > 0 ? pct_rank(a.q, n) : 0;
    const uint32_t incl = scan256(sum, s_wsum);
    if (tid == 0) s_g = -1;
    __syncthreads();
    if (n > 0 && (int64_t)(incl - sum) < k && k <= (int64_t)incl) { s_g = tid; s_below = incl - sum; }
    __syncthreads();
    if (tid < 64) {   // the crossing group's bins, one lane each
        const int g = s_g;
        int32_t bin = -1, rin = 0;
        if (g >= 0) {
            const uint32_t c = tid < per ? h[g * per + tid] : 0u;
            uint32_t in = c;
            for (int o = 1; o < per; o <<= 1) {
                const uint32_t up = __shfl_up(in, o);
                if (tid >= o) in += up;
            }
            const int64_t kk = k - s_below;
            const bool mine = tid < per && (int64_t)(in - c) < kk && kk <= (int64_t)in;
            const uint64_t m = __ballot(mine);
            const int who = m ? __ffsll((unsigned long long)m) - 1 : 0;
            const uint32_t before = __shfl(in - c, who);
            bin = g * per + who;
            rin = (int32_t)(kk - before);
        }
        if (tid == 0) {
            a.st[s].bin[j] = bin;
            a.st[s].rank_in_bin[j] = rin;
        }
    }
}

template <int V>
__global__ __launch_bounds__(FT) void k_fw_collect(FwArgs a) {
    const int64_t s = blockIdx.y;
    const int b0 = a.st[s].bin[0], b1 = a.st[s].bin[1];
    const float* hs = a.hstore + s * 2 * a.n_px;
    const int64_t nq = a.n_px / V;
    for (int64_t q = blockIdx.x * (int64_t)FT + threadIdx.x; q < nq; q += (int64_t)gridDim.x * FT) {
        float v0[V], v1[V];
        Vec<V>::load(hs + q * V, v0);
        Vec<V>::load(hs + a.n_px + q * V, v1);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const uint64_t i = (uint64_t)(q * V + k);
            if (!(__float_as_uint(v0[k]) >> 31) && coarse_bin(v0[k]) == b0) {
                const uint32_t slot = atomicAdd(&a.st[s].n_cand[0], 1u);
                if (slot < CAP) a.cand[(s * 2) * CAP + slot] = ((uint64_t)__float_as_uint(v0[k]) << 32) | i;
            }
            if (!(__float_as_uint(v1[k]) >> 31) && coarse_bin(v1[k]) == b1) {
                const uint32_t slot = atomicAdd(&a.st[s].n_cand[1], 1u);
                if (slot < CAP) a.cand[(s * 2 + 1) * CAP + slot] = ((uint64_t)__float_as_uint(v1[k]) << 32) | i;
            }
        }
    }
}

// Exact selection for one (sample, stain): a radix selection (four 8-bit digits, most significant
// first) of the rank among the candidate values (non-negative floats order like their bit patterns),
// then the smallest index holding the selected value.  The candidates are every non-white pixel of
// the coarse bin that holds the rank, so they hold every pixel of that value.  If the list
// overflowed, the same selection runs over all of the sample's non-white values.
// (blockDim.x >= 256; the digit holding rank kk is found by a parallel prefix sum of the 256 counts)
template <typename Get>
__device__ uint32_t radix_select(int64_t n_items, Get get, int64_t k, uint32_t* s_h, uint32_t* s_wsum, int* s_misc) {
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t prefix = 0, pmask = 0;
    int64_t kk = k;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += blockDim.x) s_h[b] = 0;
        __syncthreads();
        for (int64_t i = tid; i < n_items; i += blockDim.x) {
            uint32_t u;
            if (get(i, u) && (u & pmask) == prefix) atomicAdd(&s_h[(u >> shift) & 255], 1u);
        }
        __syncthreads();
        uint32_t cnt = 0, incl = 0;
        if (tid < 256) {
            cnt = s_h[tid];
            incl = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t up = __shfl_up(incl, o);
                if (lane >= o) incl += up;
            }
            if (lane == 63) s_wsum[tid >> 6] = incl;
        }
        __syncthreads();
        if (tid < 256) {
            for (int w = 0; w < (tid >> 6); ++w) incl += s_wsum[w];
            const uint32_t excl = incl - cnt;
            if ((int64_t)excl < kk && kk <= (int64_t)incl) {   // exactly one digit holds rank kk
                s_misc[0] = tid;
                s_misc[1] = (int)(kk - excl);
            }
        }
        __syncthreads();
        prefix |= (uint32_t)s_misc[0] << shift;
        pmask |= 255u << shift;
        kk = s_misc[1];
        __syncthreads();
    }
    return prefix;
}

__global__ __launch_bounds__(1024) void k_fw_select(FwArgs a) {
    __shared__ uint32_t s_h[256];
    __shared__ uint32_t s_wsum[4];
    __shared__ int s_misc[2];
    const int64_t s = blockIdx.x >> 1;
    const int j = blockIdx.x & 1;
    const int tid = threadIdx.x;
    SampleState& st = a.st[s];
    const int64_t n = st.n_tissue;
    float P = 0.0f;
    int64_t sel = -1;
    if (n > 0) {
        const uint32_t nc = st.n_cand[j];
        uint32_t bits;
        if (nc <= (uint32_t)CAP) {
            const uint64_t* cand = a.cand + (s * 2 + j) * CAP;
            bits = radix_select((int64_t)nc, [&](int64_t i, uint32_t& u) { u = (uint32_t)(cand[i] >> 32); return true; },
                                (int64_t)st.rank_in_bin[j], s_h, s_wsum, s_misc);
            if (tid == 0) s_misc[0] = 0x7FFFFFFF;
            __syncthreads();
            for (int i = tid; i < (int)nc; i += blockDim.x)
                if ((uint32_t)(cand[i] >> 32) == bits) atomicMin(&s_misc[0], (int)(uint32_t)cand[i]);
        } else {
            const float* hs = a.hstore + (s * 2 + j) * a.n_px;
            bits = radix_select(a.n_px, [&](int64_t i, uint32_t& u) { u = __float_as_uint(hs[i]); return !(u >> 31); },
                                pct_rank(a.q, n), s_h, s_wsum, s_misc);
            if (tid == 0) s_misc[0] = 0x7FFFFFFF;
            __syncthreads();
            for (int64_t i = tid; i < a.n_px; i += blockDim.x)
                if (__float_as_uint(hs[i]) == bits) atomicMin(&s_misc[0], (int)i);
        }
        __syncthreads();
        P = __uint_as_float(bits);
        sel = s_misc[0];
    }
    if (tid == 0) {
        int fl = n == 0 ? SPCN_FLAG_NO_TISSUE : 0;
        if (n > 0 && !(P > 0.0f)) fl |= SPCN_FLAG_BIN0;
        Basis64 B;
        derive_basis(a.w_src + s * a.w_src_stride, a.lambda, B);
        if (!B.ok) fl |= SPCN_FLAG_BASIS;
        const float S = a.scale_tgt[s * a.scale_stride + j];
        const float sj = (fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0)) ? 1.0f : S / P;
        st.P[j] = P; st.s[j] = sj; st.sel[j] = sel; st.flags[j] = fl;
        const float* wt = a.w_tgt + s * a.w_tgt_stride;
        for (int c = 0; c < 3; ++c) {
            st.M[c][j] = (float)(kLog2e * (double)wt[c + 3 * j] * (double)sj);
            if (j == 0) st.L[c] = a.log2io[c];
        }
        if (a.p99_out) a.p99_out[2 * s + j] = P;
        if (a.scale_out) a.scale_out[2 * s + j] = sj;
        if (a.sel_idx) a.sel_idx[2 * s + j] = sel;
        if (a.flags_out) a.flags_out[2 * s + j] = fl;
    }
}

template <int V>
__global__ __launch_bounds__(FT) void k_fw_recon(FwArgs a) {
    const int64_t s = blockIdx.y;
    const SampleState& st = a.st[s];
    float M[3][2], L[3];
    for (int c = 0; c < 3; ++c) { M[c][0] = st.M[c][0]; M[c][1] = st.M[c][1]; L[c] = st.L[c]; }
    const float* hs = a.hstore + s * 2 * a.n_px;
    float* y = a.y + s * 3 * a.n_px;
    const int64_t nq = a.n_px / V;
    for (int64_t q = blockIdx.x * (int64_t)FT + threadIdx.x; q < nq; q += (int64_t)gridDim.x * FT) {
        const int64_t i = q * V;
        float h0[V], h1[V];
        Vec<V, false>::load(hs + i, h0);
        Vec<V, false>::load(hs + a.n_px + i, h1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float yc[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                float z = fmaf(-M[c][0], fabsf(h0[k]), L[c]);
                z = fmaf(-M[c][1], fabsf(h1[k]), z);
                yc[k] = __builtin_amdgcn_exp2f(z);
            }
            Vec<V, false>::store(y + c * a.n_px + i, yc);
        }
    }
}

// ------------------------------------------------------------------ backward

struct BwArgs {
    const float* x; int64_t n, n_px;
    const float* w_src; int64_t w_src_stride;
    const float* w_tgt; int64_t w_tgt_stride;
    const float* scale_tgt; int64_t scale_stride;
    float i0[3], i0_out[3], lambda;
    float log2i0[3], log2io[3];   // log2 of i0 and i0_out (host-computed)
    int32_t white_sum;
    const float* p99; const int64_t* sel; const int32_t* flags;
    const float* gy;
    float* gx; float* gw; float* gs;
    double* partial;        // [n][blocks][8]
    double* per_sample;     // [n][8]: each sample's dWt (6) and dscale (2), for parameters shared by the batch
};

struct BwConsts {
    float s[2];
    float wt[6];
    float log2io[3];
};

__device__ inline void bw_consts(const BwArgs& a, int64_t s, BwConsts& K) {
    for (int j = 0; j < 2; ++j) {
        const int fl = a.flags[2 * s + j];
        const float P = a.p99[2 * s + j];
        const float S = a.scale_tgt[s * a.scale_stride + j];
        K.s[j] = (fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0)) ? 1.0f : S / P;
    }
    for (int i = 0; i < 6; ++i) K.wt[i] = a.w_tgt[s * a.w_tgt_stride + i];
    for (int c = 0; c < 3; ++c) K.log2io[c] = a.log2io[c];
}

// Gradient of one pixel w.r.t. its inputs given hbar (both stains), on its active set.
__device__ __forceinline__ void pixel_vjp(const F32Basis& F, const Px& p, float hb0, float hb1, float x0, float x1,
                                          float x2, float g[3]) {
    float z0 = 0.0f, z1 = 0.0f;
    const bool a0 = p.h0 > 0.0f, a1 = p.h1 > 0.0f;
    if (a0 && a1) {
        z0 = (F.g11 * hb0 - F.g01 * hb1) * F.r_det;
        z1 = (F.g00 * hb1 - F.g01 * hb0) * F.r_det;
    } else if (a0) {
        z0 = hb0 * F.r00;
    } else if (a1) {
        z1 = hb1 * F.r11;
    }
    const float xs[3] = {x0, x1, x2};
    for (int c = 0; c < 3; ++c) {
        const float vbar = F.w[c] * z0 + F.w[c + 3] * z1;
        g[c] = p.live[c] ? -vbar * __builtin_amdgcn_rcpf(xs[c]) : 0.0f;   // live: x_c above the real 1/255
    }
}

template <int V>
__global__ __launch_bounds__(FT) void k_bw_main(BwArgs a) {
    __shared__ F32Basis F;
    __shared__ BwConsts K;
    __shared__ double s_red[FT / 64][8];
    const int64_t s = blockIdx.y;
    if (threadIdx.x == 0) {
        f32_basis(a.w_src + s * a.w_src_stride, a.lambda, a.i0, a.log2i0, F);
        bw_consts(a, s, K);
    }
    __syncthreads();
    const float* x = a.x + s * 3 * a.n_px;
    const float* gy = a.gy + s * 3 * a.n_px;
    float* gx = a.gx + s * 3 * a.n_px;
    // dWt[c][j] at c + 3 j, then ds0, ds1: FP32 over this thread's few pixels, FP64 from there on
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t nq = a.n_px / V;
    for (int64_t q = blockIdx.x * (int64_t)FT + threadIdx.x; q < nq; q += (int64_t)gridDim.x * FT) {
        const int64_t i = q * V;
        float xv[3][V], gv[3][V], out[3][V];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Vec<V>::load(x + c * a.n_px + i, xv[c]);
            Vec<V>::load(gy + c * a.n_px + i, gv[c]);
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            Px p;
            solve_px(F, xv[0][k], xv[1][k], xv[2][k], a.white_sum, p);
            float ub[3];
            float hb0 = 0.0f, hb1 = 0.0f;
            for (int c = 0; c < 3; ++c) {
                float z = fmaf(-K.wt[c] * K.s[0] * (float)kLog2e, p.h0, K.log2io[c]);
                z = fmaf(-K.wt[c + 3] * K.s[1] * (float)kLog2e, p.h1, z);
                const float y = __builtin_amdgcn_exp2f(z);
                ub[c] = -y * gv[c][k];
                acc[c] = fmaf(ub[c] * K.s[0], p.h0, acc[c]);
                acc[c + 3] = fmaf(ub[c] * K.s[1], p.h1, acc[c + 3]);
                hb0 = fmaf(K.wt[c], ub[c], hb0);
                hb1 = fmaf(K.wt[c + 3], ub[c], hb1);
            }
            acc[6] = fmaf(hb0, p.h0, acc[6]);
            acc[7] = fmaf(hb1, p.h1, acc[7]);
            float g[3];
            pixel_vjp(F, p, K.s[0] * hb0, K.s[1] * hb1, xv[0][k], xv[1][k], xv[2][k], g);
            for (int c = 0; c < 3; ++c) out[c][k] = g[c];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) Vec<V>::store(gx + c * a.n_px + i, out[c]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = 0; q < 8; ++q) {
        double v = (double)acc[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s_red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int w = 0; w < FT / 64; ++w) t += s_red[w][threadIdx.x];
        a.partial[(s * gridDim.x + blockIdx.x) * 8 + threadIdx.x] = t;
    }
}

__global__ __launch_bounds__(64) void k_bw_reduce(BwArgs a, int nblk) {
    __shared__ double s_part[8][8];   // [block group][quantity]
    __shared__ double s_t[8];
    const int64_t s = blockIdx.x;
    {   // fixed association: group g sums blocks g, g + 8, ...; then the groups in order
        const int q = threadIdx.x & 7, g = threadIdx.x >> 3;
        double v = 0.0;
        for (int b = g; b < nblk; b += 8) v += a.partial[(s * nblk + b) * 8 + q];
        s_part[g][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double v = 0.0;
        for (int g = 0; g < 8; ++g) v += s_part[g][threadIdx.x];
        s_t[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[8];
    for (int q = 0; q < 8; ++q) t[q] = s_t[q];
    for (int i = 0; i < 6; ++i) {
        if (a.w_tgt_stride) a.gw[6 * s + i] = (float)t[i];
        else a.per_sample[8 * s + i] = t[i];
    }
    F32Basis F;
    f32_basis(a.w_src + s * a.w_src_stride, a.lambda, a.i0, a.log2i0, F);
    BwConsts K;
    bw_consts(a, s, K);
    const float* x = a.x + s * 3 * a.n_px;
    float* gx = a.gx + s * 3 * a.n_px;
    for (int j = 0; j < 2; ++j) {
        const int fl = a.flags[2 * s + j];
        const bool scaled = !(fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0));
        const float P = a.p99[2 * s + j];
        const double gsj = scaled ? t[6 + j] / (double)P : 0.0;
        if (a.scale_stride) a.gs[2 * s + j] = (float)gsj;
        else a.per_sample[8 * s + 6 + j] = gsj;
        if (!scaled) continue;
        // the percentile is the density of the selected pixel: its adjoint joins that pixel's hbar
        const double Pbar = -((double)K.s[j] / (double)P) * t[6 + j];
        const int64_t i = a.sel[2 * s + j];
        if (i < 0 || i >= a.n_px) continue;
        Px p;
        solve_px(F, x[i], x[a.n_px + i], x[2 * a.n_px + i], a.white_sum, p);
        float g[3];
        pixel_vjp(F, p, j == 0 ? (float)Pbar : 0.0f, j == 1 ? (float)Pbar : 0.0f, x[i], x[a.n_px + i],
                  x[2 * a.n_px + i], g);
        for (int c = 0; c < 3; ++c) gx[c * a.n_px + i] += g[c];
    }
}

// A target basis or scale shared by the whole batch (stride 0) gets the sum of the per-sample
// gradients in FP64, in a fixed association (deterministic): thread t of quantity q's 64 threads
// sums samples t, t + 64, ... in order, then the 64 partial sums are added pairwise in LDS.
__global__ __launch_bounds__(512) void k_bw_shared(BwArgs a) {
    __shared__ double s_v[8][64];
    const int q = threadIdx.x >> 6, t = threadIdx.x & 63;
    double v = 0.0;
    for (int64_t s = t; s < a.n; s += 64) v += a.per_sample[8 * s + q];
    s_v[q][t] = v;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
        if (t < h) s_v[q][t] += s_v[q][t + h];
        __syncthreads();
    }
    if (t == 0) {
        if (q < 6 && !a.w_tgt_stride) a.gw[q] = (float)s_v[q][0];
        if (q >= 6 && !a.scale_stride) a.gs[q - 6] = (float)s_v[q][0];
    }
}

int blocks_per_sample(int64_t n_px, int64_t n, const DevInfo& dev) {
    int64_t want = (n_px + FT * 16 - 1) / (FT * 16);   // about 16 pixels per thread
    int64_t cap = ((int64_t)dev.cus * 8 + n - 1) / n;
    int64_t b = want < cap ? want : cap;
    if (b > BLOCKS_PER_SAMPLE_MAX) b = BLOCKS_PER_SAMPLE_MAX;
    return (int)(b < 1 ? 1 : b);
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

size_t f32_forward_workspace_bytes(int64_t n_px, int64_t n) {
    if (n_px <= 0 || n <= 0) return 0;
    return a256((size_t)n * 2 * n_px * sizeof(float)) + a256((size_t)n * 2 * NBIN * sizeof(uint32_t)) +
           a256((size_t)n * sizeof(SampleState)) + a256((size_t)n * 2 * CAP * sizeof(uint64_t));
}

size_t f32_backward_workspace_bytes(int64_t n_px, int64_t n) {
    if (n_px <= 0 || n <= 0) return 0;
    (void)n_px;
    return a256((size_t)n * BLOCKS_PER_SAMPLE_MAX * 8 * sizeof(double)) + a256((size_t)n * 8 * sizeof(double));
}

hipError_t launch_forward_f32(const F32Args& g, const ParamsK& pk, float* y, float* p99_out, float* scale_out,
                              int64_t* sel_idx, int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s) {
    FwArgs a{};
    a.x = g.x; a.n = g.n; a.n_px = g.n_px;
    a.w_src = g.w_src; a.w_src_stride = g.w_src_stride; a.w_tgt = g.w_tgt; a.w_tgt_stride = g.w_tgt_stride;
    a.scale_tgt = g.scale_tgt; a.scale_stride = g.scale_stride;
    for (int c = 0; c < 3; ++c) {
        a.i0[c] = pk.i0[c]; a.i0_out[c] = g.i0_out[c];
        a.log2i0[c] = (float)std::log2((double)pk.i0[c]); a.log2io[c] = (float)std::log2((double)g.i0_out[c]);
    }
    a.lambda = pk.lambda; a.white_sum = pk.white_sum; a.q = pk.q64;
    uint8_t* p = static_cast<uint8_t*>(ws);
    a.hstore = reinterpret_cast<float*>(p); p += a256((size_t)g.n * 2 * g.n_px * sizeof(float));
    a.chist = reinterpret_cast<uint32_t*>(p); p += a256((size_t)g.n * 2 * NBIN * sizeof(uint32_t));
    a.st = reinterpret_cast<SampleState*>(p); p += a256((size_t)g.n * sizeof(SampleState));
    a.cand = reinterpret_cast<uint64_t*>(p);
    a.y = y; a.p99_out = p99_out; a.scale_out = scale_out; a.sel_idx = sel_idx; a.flags_out = flags_out;
    const int bps = blocks_per_sample(g.n_px, g.n, dev);
    const dim3 grid(bps, (unsigned)g.n);
    // planes of n_px floats: 16-byte accesses when every plane starts 16-byte aligned
    const bool v4 = g.n_px % 4 == 0 && aligned16(g.x) && aligned16(y) && aligned16(a.hstore);
    hipLaunchKernelGGL(k_fw_clear, dim3(dev.cus), dim3(256), 0, s, a);
    const dim3 grid_d((bps + 1) / 2, (unsigned)g.n);   // half the workgroups: half the histogram merges
    if (v4) hipLaunchKernelGGL(k_fw_dens<4>, grid_d, dim3(FT), 0, s, a);
    else hipLaunchKernelGGL(k_fw_dens<1>, grid_d, dim3(FT), 0, s, a);
    hipLaunchKernelGGL(k_fw_bin, dim3((unsigned)(2 * g.n)), dim3(FT), 0, s, a);
    if (v4) hipLaunchKernelGGL(k_fw_collect<4>, grid, dim3(FT), 0, s, a);
    else hipLaunchKernelGGL(k_fw_collect<1>, grid, dim3(FT), 0, s, a);
    hipLaunchKernelGGL(k_fw_select, dim3((unsigned)(2 * g.n)), dim3(1024), 0, s, a);
    if (v4) hipLaunchKernelGGL(k_fw_recon<4>, grid, dim3(FT), 0, s, a);
    else hipLaunchKernelGGL(k_fw_recon<1>, grid, dim3(FT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_backward_f32(const F32Args& g, const ParamsK& pk, const float* p99, const int64_t* sel_idx,
                               const int32_t* flags, const float* grad_y, float* grad_x, float* grad_w_tgt,
                               float* grad_scale, void* ws, const DevInfo& dev, hipStream_t s) {
    BwArgs a{};
    a.x = g.x; a.n = g.n; a.n_px = g.n_px;
    a.w_src = g.w_src; a.w_src_stride = g.w_src_stride; a.w_tgt = g.w_tgt; a.w_tgt_stride = g.w_tgt_stride;
    a.scale_tgt = g.scale_tgt; a.scale_stride = g.scale_stride;
    for (int c = 0; c < 3; ++c) {
        a.i0[c] = pk.i0[c]; a.i0_out[c] = g.i0_out[c];
        a.log2i0[c] = (float)std::log2((double)pk.i0[c]); a.log2io[c] = (float)std::log2((double)g.i0_out[c]);
    }
    a.lambda = pk.lambda; a.white_sum = pk.white_sum;
    a.p99 = p99; a.sel = sel_idx; a.flags = flags; a.gy = grad_y;
    a.gx = grad_x; a.gw = grad_w_tgt; a.gs = grad_scale;
    a.partial = static_cast<double*>(ws);
    a.per_sample = reinterpret_cast<double*>(static_cast<uint8_t*>(ws) +
                                             a256((size_t)g.n * BLOCKS_PER_SAMPLE_MAX * 8 * sizeof(double)));
    const int bps = blocks_per_sample(g.n_px, g.n, dev);
    const bool v4 = g.n_px % 4 == 0 && aligned16(g.x) && aligned16(grad_y) && aligned16(grad_x);
    if (v4) hipLaunchKernelGGL(k_bw_main<4>, dim3(bps, (unsigned)g.n), dim3(FT), 0, s, a);
    else hipLaunchKernelGGL(k_bw_main<1>, dim3(bps, (unsigned)g.n), dim3(FT), 0, s, a);
    hipLaunchKernelGGL(k_bw_reduce, dim3((unsigned)g.n), dim3(64), 0, s, a, bps);
    if (g.w_tgt_stride == 0 || g.scale_stride == 0) hipLaunchKernelGGL(k_bw_shared, dim3(1), dim3(512), 0, s, a);
    return hipGetLastError();
}

}  // namespace spcn
