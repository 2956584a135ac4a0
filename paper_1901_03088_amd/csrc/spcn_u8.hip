// spcn_u8.hip -- fused SPCN normalisation of one uint8 RGB image on gfx950 (Eqs. 1-4, Sec. 2.1;
// the non-white percentile of Sec. 3.1 item 2).
//
//   k_pass1   reads 3 B/px: densities of every non-white pixel, exact 2 x 256 histogram
//             (one workgroup per CU, a contiguous chunk each; see spcn_passes.hpp);
//   k_pass2   every workgroup recomputes the percentile from the histogram in its prologue (no
//             separate finalisation launch), then re-reads 3 B/px, recolours and writes 3 B/px;
//   k_pass1d  pass 1 writing the FP32 densities as well (spcn_densities with h_out);
//   k_finalize percentile + flags of a histogram for spcn_densities;
//   k_u8_setup / k_range_check  histogram range kept on the device: the range of the call, and one
//             automatic retry at twice a stain's range when its percentile lands in the open last
//             bin (a second pass-1 launch that ends at once unless the check asked for it).
//
// Kernel variants (table replication, histogram columns, workgroups per CU) are selected at run
// time through spcn_set_option; all variants compute identical results.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int P1_THREADS = 1024;
constexpr int P2_UNROLL = 4;      // units per thread and iteration of the chunked pass 2
// Grid-stride pass 2: 16 units (192 bytes) per thread and tile keep enough loads in flight at the
// occupancy its registers allow (measured on the slide: 4 -> 2.43 ms, 8 -> 2.40, 16 -> 2.34, 24 the
// same as 16, 32 spills); 1024-thread workgroups keep 4.
__host__ __device__ constexpr int p2g_unroll(int threads) { return threads >= 1024 ? 4 : 16; }

struct P1Args {
    const uint8_t* src;
    int64_t n_px;
    const float* w;
    P1Params pp;
    unsigned long long* hist;      // global [2][256]
    int64_t scatter, step;         // tile permutation of the grid-stride kernels (p1f_tiles)
    const int32_t* gate;           // if non-NULL, the launch does nothing unless *gate != 0
};

__device__ __forceinline__ bool gated_off(const int32_t* gate) { return gate && *gate == 0; }

// WAVES: minimum waves per SIMD the compiler must allow (register budget); 4 = one workgroup per CU,
// 8 = two (the small-LDS variants).
template <int COPIES, int COLS, int UNROLL, int WAVES>
__global__ __launch_bounds__(P1_THREADS, WAVES) void k_pass1(const P1Args a) {
    __shared__ P1Lds<COPIES, COLS> S;
    if (gated_off(a.gate)) return;
    const P1Params pp = p1_resolve(a.pp);
    p1_setup(S, a.w, pp, true);
    const int64_t n_units = a.n_px >> 2;
    const int64_t per = (n_units + gridDim.x - 1) / gridDim.x;
    const int64_t ubeg = min(n_units, (int64_t)blockIdx.x * per);
    const int cnt = (int)(min(n_units, ubeg + per) - ubeg);
    p1_chunk<COPIES, COLS, UNROLL>(S, pp, chunk_rsrc(a.src, ubeg, cnt), a.src + 12 * ubeg, cnt, threadIdx.x,
                                      P1_THREADS);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        p1_tail(S, pp, a.src + 12 * n_units, (int)(a.n_px - 4 * n_units));
    p1_merge(S, a.hist);
}

// Range and retry words of the single-image path, kept in the caller's workspace after the histogram.
struct U8Ctl {
    float range[2];     // histogram range of each stain for this call
    int32_t retry;      // bit j: stain j's range was doubled and pass 1 must run again
    int32_t pad;
};

// Zeroes the histogram and settles the call's range (device value if given, else the host one).
__global__ __launch_bounds__(256) void k_u8_setup(uint64_t* hist, U8Ctl* ctl, const float* range_dev, float hh0,
                                                  float hh1) {
    for (int i = threadIdx.x; i < 2 * kHistBins; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) {
        ctl->range[0] = resolve_range(range_dev, hh0);
        ctl->range[1] = resolve_range(range_dev ? range_dev + 1 : nullptr, hh1);
        ctl->retry = 0;
    }
}

// Eq. 3's percentile of each stain from the histogram; a stain whose percentile lies in the open
// last bin gets twice its range (up to 2^8) and the histogram is cleared for a second pass 1.
// range_out (or NULL) receives the settled range.
__global__ __launch_bounds__(256) void k_range_check(uint64_t* hist, U8Ctl* ctl, double q, float* range_out) {
    __shared__ FinalShared F;
    __shared__ int bits;
    const float hh[2] = {ctl->range[0], ctl->range[1]};
    block_percentiles(hist, q, hh, F);
    if (threadIdx.x == 0) {
        int b = 0;
        for (int j = 0; j < 2; ++j)
            if (F.kstar[j] == kHistBins - 1 && hh[j] < 256.0f) b |= 1 << j;
        bits = b;
    }
    __syncthreads();
    if (bits) {
        for (int i = threadIdx.x; i < 2 * kHistBins; i += blockDim.x) hist[i] = 0;
        if (threadIdx.x == 0) {
            for (int j = 0; j < 2; ++j)
                if (bits & (1 << j)) ctl->range[j] = 2.0f * hh[j];
            ctl->retry = bits;
        }
    }
    if (range_out && threadIdx.x < 2) range_out[threadIdx.x] = (bits >> threadIdx.x & 1) ? 2.0f * hh[threadIdx.x] : hh[threadIdx.x];
}

__device__ __forceinline__ int retry_flag(const int32_t* retry, int j) {
    return (retry && (*retry >> j) & 1) ? SPCN_FLAG_RANGE_RETRY : 0;
}

__global__ __launch_bounds__(256) void k_finalize(const uint64_t* hist, double q, const float* range, float hh0,
                                                  float hh1, const int32_t* retry, const float* w, float lambda,
                                                  float* p99_out, int32_t* flags_out, float* range_out) {
    __shared__ FinalShared F;
    __shared__ int basis_ok;
    const float hh[2] = {resolve_range(range, hh0), resolve_range(range ? range + 1 : nullptr, hh1)};
    if (threadIdx.x == 0) { Basis64 B; derive_basis(w, lambda, B); basis_ok = B.ok; }
    block_percentiles(hist, q, hh, F);
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        if (p99_out) p99_out[j] = (float)F.P[j];
        if (flags_out) flags_out[j] = stain_flags(F, j, basis_ok) | retry_flag(retry, j);
        if (range_out) range_out[j] = hh[j];
    }
}

__global__ void k_zero_u64(uint64_t* p, int n) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) p[i] = 0;
}

// Pass 1 with the FP32 densities of every pixel (Eq. 2 with W fixed), planar [2][n_px]: the exact
// histogram of k_pass1g's wide layout and, from the same read of each unit, the densities -- from the
// fixed-point candidate sums of the histogram when u = 16 (p1f_tiles_dens16), else from the FP32
// tables of the recolour pass -- one 16-byte store per unit and stain (3 B/px read, 8 B/px
// written).  One 1024-thread workgroup per CU, the tiles in the scattered order of k_pass1g.
template <int UNROLL>
__global__ __launch_bounds__(1024, 4) void k_pass1d(const P1Args a, float* h_out) {
    __shared__ P1FLds<true> S;
    __shared__ P2Lds<1> T;
    __shared__ float s_a[2];
    const P1Params pp = p1_resolve(a.pp);
    p1f_setup(S, a.w, pp, true);
    p2_tables(T, S.B, pp.i0);
    if (threadIdx.x == 0) { s_a[0] = (float)S.B.a[0]; s_a[1] = (float)S.B.a[1]; }
    __syncthreads();
    RecolourConsts K{};
    K.a0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_a[0])));
    K.a1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_a[1])));
    const int64_t n_units = a.n_px >> 2;
    const bool u16 = S.shift == 16;
    if (u16)
        p1f_tiles_dens16<UNROLL>(S, pp, a.src, n_units, h_out, a.n_px, threadIdx.x, 1024, a.scatter, a.step);
    else
        p1f_tiles_dens<true, UNROLL, false>(S, T, K, pp, a.src, n_units, h_out, a.n_px, threadIdx.x, 1024, a.scatter,
                                           a.step);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int tail = (int)(a.n_px - 4 * n_units);
        const uint8_t* px = a.src + 12 * n_units;
        p1f_tail(S, pp, px, tail);
        const P1FLane L = p1f_lane<true>(0, pp.white_sum);
        for (int i = 0; i < tail; ++i) {
            float h0, h1;
            if (u16) {   // the densities from the fixed-point sums, as in the body
                int32_t y0, y1;
                p1f_sums(S, px[3 * i], px[3 * i + 1], px[3 * i + 2], L.r16, y0, y1);
                h0 = fmaxf(0.0f, (float)(y0 + kGuardUnits) * (float)((double)pp.hist_hi[0] / 16777216.0));
                h1 = fmaxf(0.0f, (float)(y1 + kGuardUnits) * (float)((double)pp.hist_hi[1] / 16777216.0));
            } else {
                p2_densities(T, 0u, K, px[3 * i], px[3 * i + 1], px[3 * i + 2], h0, h1);
            }
            h_out[4 * n_units + i] = h0;
            h_out[a.n_px + 4 * n_units + i] = h1;
        }
    }
    p1f_merge(S, a.hist);
}

struct P2Args {
    const uint8_t* src;
    uint8_t* out;
    int64_t n_px;
    const float* w_src;
    const float* w_tgt;
    const float* scale_tgt;
    float i0[3];
    float i0_out[3];
    float lambda;
    float hist_hi[2];
    const float* range;        // device range [2] replacing hist_hi (resolve_range), or NULL
    const int32_t* retry;      // retry bits of the call (SPCN_FLAG_RANGE_RETRY), or NULL
    double q;
    const uint64_t* hist;
    const float* p99_in;       // given source percentiles [2] (then hist is not read), or NULL
    float* p99_out;
    float* scale_out;
    int32_t* flags_out;
    float* range_out;          // [2] range used, or NULL
};

// Prologue of every pass-2 workgroup: tables, percentile and recolouring constants (block 0 also
// writes the statistics).  Ends with a barrier.
template <int COPIES>
__device__ void p2_prologue(const P2Args& a, P2Lds<COPIES>& T, FinalShared& F, Basis64& B, RecolourConsts& K) {
    if (threadIdx.x == 0) derive_basis(a.w_src, a.lambda, B);
    __syncthreads();
    p2_tables(T, B, a.i0);
    const float hh[2] = {resolve_range(a.range, a.hist_hi[0]), resolve_range(a.range ? a.range + 1 : nullptr, a.hist_hi[1])};
    if (a.p99_in) {
        if (threadIdx.x < 2) F.P[threadIdx.x] = (double)a.p99_in[threadIdx.x];
    } else {
        block_percentiles(a.hist, a.q, hh, F);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[2];
        int fl[2];
        for (int j = 0; j < 2; ++j) {
            // a given percentile that is not > 0 keeps the stain unscaled, like a bin-0 percentile
            fl[j] = (a.p99_in ? ((F.P[j] > 0.0 ? 0 : SPCN_FLAG_BIN0) | (B.ok ? 0 : SPCN_FLAG_BASIS))
                              : stain_flags(F, j, B.ok) | retry_flag(a.retry, j)) |
                    scale_flag(a.scale_tgt[j]);
            s[j] = stain_scale((double)a.scale_tgt[j], F.P[j], fl[j]);
        }
        make_recolour(K, a.w_tgt, s, a.i0_out, B);
        if (blockIdx.x == 0) {
            for (int j = 0; j < 2; ++j) {
                if (a.p99_out) a.p99_out[j] = (float)F.P[j];
                if (a.scale_out) a.scale_out[j] = (float)s[j];
                if (a.flags_out) a.flags_out[j] = fl[j];
                if (a.range_out) a.range_out[j] = hh[j];
            }
        }
    }
    __syncthreads();
}

template <int COPIES, int THREADS>
__global__ __launch_bounds__(THREADS) void k_pass2(const P2Args a) {
    __shared__ P2Lds<COPIES> T;
    __shared__ FinalShared F;
    __shared__ Basis64 B;
    __shared__ RecolourConsts K;
    p2_prologue(a, T, F, B, K);
    const RecolourConsts Kr = K;
    const int64_t n_units = a.n_px >> 2;
    const int64_t per = (n_units + gridDim.x - 1) / gridDim.x;
    const int64_t ubeg = min(n_units, (int64_t)blockIdx.x * per);
    const int cnt = (int)(min(n_units, ubeg + per) - ubeg);
    p2_chunk<COPIES, P2_UNROLL>(T, Kr, chunk_rsrc(a.src, ubeg, cnt), chunk_rsrc(a.out, ubeg, cnt), cnt, threadIdx.x,
                                THREADS);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        p2_tail(T, Kr, a.src + 12 * n_units, a.out + 12 * n_units, (int)(a.n_px - 4 * n_units));
}

// Grid-stride pass 2 (the grid sweeps the image front to back together).
template <int COPIES, int THREADS>
__global__ __launch_bounds__(THREADS) void k_pass2g(const P2Args a) {
    __shared__ P2Lds<COPIES> T;
    __shared__ FinalShared F;
    __shared__ Basis64 B;
    __shared__ RecolourConsts K;
    p2_prologue(a, T, F, B, K);
    const RecolourConsts Kr = K;
    const int64_t n_units = a.n_px >> 2;
    p2_tiles<COPIES, p2g_unroll(THREADS)>(T, Kr, a.src, a.out, n_units, threadIdx.x, THREADS);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        p2_tail(T, Kr, a.src + 12 * n_units, a.out + 12 * n_units, (int)(a.n_px - 4 * n_units));
}

// Grid-stride pass 1 with the byte-permute layouts (see p1f_units); same counts as k_pass1.
// WIDE: one 1024-thread workgroup per CU; narrow: two 768-thread workgroups per CU.
template <bool WIDE, int THREADS, int UNROLL, int WAVES>
__global__ __launch_bounds__(THREADS, WAVES) void k_pass1g(const P1Args a) {
    __shared__ P1FLds<WIDE> S;
    if (gated_off(a.gate)) return;
    const P1Params pp = p1_resolve(a.pp);
    p1f_setup(S, a.w, pp, true);
    const int64_t n_units = a.n_px >> 2;
    if (S.shift == 16)
        p1f_tiles<WIDE, UNROLL, true>(S, pp, a.src, n_units, threadIdx.x, THREADS, a.scatter, a.step);
    else
        p1f_tiles<WIDE, UNROLL, false>(S, pp, a.src, n_units, threadIdx.x, THREADS, a.scatter, a.step);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        p1f_tail(S, pp, a.src + 12 * n_units, (int)(a.n_px - 4 * n_units));
    p1f_merge(S, a.hist);
}

template <int COPIES, int COLS, int UNROLL, int WAVES>
hipError_t run_pass1(const P1Args& a, const DevInfo& dev, hipStream_t s) {
    int64_t units = a.n_px >> 2;
    int64_t want = (units + (int64_t)P1_THREADS * UNROLL - 1) / ((int64_t)P1_THREADS * UNROLL);
    int64_t cap = (int64_t)dev.cus * (WAVES / 4);
    int grid = (int)(want < 1 ? 1 : (want < cap ? want : cap));
    hipLaunchKernelGGL((k_pass1<COPIES, COLS, UNROLL, WAVES>), dim3(grid), dim3(P1_THREADS), 0, s, a);
    return hipGetLastError();
}

template <bool WIDE, int THREADS, int UNROLL, int WAVES>
hipError_t run_pass1g(const P1Args& a, int per_cu, const DevInfo& dev, hipStream_t s) {
    int64_t tiles = ((a.n_px >> 2) + (int64_t)THREADS * UNROLL - 1) / ((int64_t)THREADS * UNROLL);
    int64_t cap = (int64_t)dev.cus * per_cu;
    int grid = (int)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
    P1Args b = a;
    b.scatter = tile_scatter(tiles, grid);
    b.step = tiles > 0 ? ((int64_t)grid * b.scatter) % tiles : 0;
    hipLaunchKernelGGL((k_pass1g<WIDE, THREADS, UNROLL, WAVES>), dim3(grid), dim3(THREADS), 0, s, b);
    return hipGetLastError();
}

template <int UNROLL>
hipError_t run_pass1d(const P1Args& a, float* h_out, const DevInfo& dev, hipStream_t s) {
    int64_t tiles = ((a.n_px >> 2) + 1024 * UNROLL - 1) / (1024 * UNROLL);
    int64_t cap = dev.cus;
    int grid = (int)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
    P1Args b = a;
    b.scatter = tile_scatter(tiles, grid);
    b.step = tiles > 0 ? ((int64_t)grid * b.scatter) % tiles : 0;
    hipLaunchKernelGGL((k_pass1d<UNROLL>), dim3(grid), dim3(1024), 0, s, b, h_out);
    return hipGetLastError();
}

template <int COPIES, int THREADS>
hipError_t run_pass2g(const P2Args& a, int blocks_per_cu, const DevInfo& dev, hipStream_t s) {
    constexpr int U = p2g_unroll(THREADS);
    int64_t tiles = ((a.n_px >> 2) + (int64_t)THREADS * U - 1) / ((int64_t)THREADS * U);
    int64_t cap = (int64_t)dev.cus * blocks_per_cu;
    int grid = (int)(tiles < 1 ? 1 : (tiles < cap ? tiles : cap));
    hipLaunchKernelGGL((k_pass2g<COPIES, THREADS>), dim3(grid), dim3(THREADS), 0, s, a);
    return hipGetLastError();
}

template <int COPIES, int THREADS>
hipError_t run_pass2(const P2Args& a, int blocks_per_cu, const DevInfo& dev, hipStream_t s) {
    int64_t units = a.n_px >> 2;
    int64_t want = (units + (int64_t)THREADS * P2_UNROLL - 1) / ((int64_t)THREADS * P2_UNROLL);
    int64_t cap = (int64_t)dev.cus * blocks_per_cu;
    int grid = (int)(want < 1 ? 1 : (want < cap ? want : cap));
    hipLaunchKernelGGL((k_pass2<COPIES, THREADS>), dim3(grid), dim3(THREADS), 0, s, a);
    return hipGetLastError();
}

}  // namespace

// ----------------------------------------------------------------------------- launchers

size_t u8_workspace_bytes() { return 2 * kHistBins * sizeof(uint64_t) + 256; }

static U8Ctl* ctl_of(void* ws) {
    return reinterpret_cast<U8Ctl*>(static_cast<uint8_t*>(ws) + 2 * kHistBins * sizeof(uint64_t));
}

static hipError_t launch_pass1(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk, uint64_t* hist,
                               const float* range, const int32_t* gate, const DevInfo& dev, hipStream_t s,
                               float* h_out = nullptr) {
    P1Args a{};
    a.src = img; a.n_px = n_px; a.w = w;
    for (int c = 0; c < 3; ++c) a.pp.i0[c] = pk.i0[c];
    a.pp.lambda = pk.lambda; a.pp.white_sum = pk.white_sum;
    a.pp.hist_hi[0] = pk.hist_hi[0]; a.pp.hist_hi[1] = pk.hist_hi[1];
    a.pp.range = range;
    a.hist = reinterpret_cast<unsigned long long*>(hist);
    a.gate = gate;
    if (h_out) return run_pass1d<2>(a, h_out, dev, s);
    switch (option(SPCN_OPT_P1_VARIANT)) {
        case 0: return run_pass1<1, 64, 4, 4>(a, dev, s);
        case 1: return run_pass1<2, 64, 4, 4>(a, dev, s);
        case 2: return run_pass1<4, 32, 4, 4>(a, dev, s);
        case 3: return run_pass1<8, 16, 4, 4>(a, dev, s);
        case 4: return run_pass1<1, 32, 2, 8>(a, dev, s);
        case 5: return run_pass1<2, 16, 2, 8>(a, dev, s);
        case 6: return run_pass1g<true, 1024, 4, 4>(a, 1, dev, s);
        case 7: return run_pass1g<true, 1024, 2, 4>(a, 1, dev, s);
        case 8: return run_pass1g<false, 768, 2, 6>(a, 2, dev, s);
        default: return run_pass1g<false, 512, 2, 4>(a, 2, dev, s);
    }
}

hipError_t launch_zero_hist(uint64_t* hist, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, hist, 2 * kHistBins);
    return hipGetLastError();
}

hipError_t launch_count(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk, uint64_t* hist,
                        const DevInfo& dev, hipStream_t s) {
    return launch_pass1(img, n_px, w, pk, hist, pk.hist_hi_dev, nullptr, dev, s);
}

// Histogram of the call with its range settled on the device: set-up, pass 1 (writing the densities
// too when h_out is given) and, with auto_range, the range check and the gated second pass 1 (the
// densities do not depend on the range).  The range and retry words are in ctl.
static hipError_t launch_hist_checked(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                                      uint64_t* hist, void* ctl_ws, const DevInfo& dev, hipStream_t s,
                                      float* h_out = nullptr, float* range_out = nullptr) {
    U8Ctl* ctl = ctl_of(ctl_ws);
    hipLaunchKernelGGL(k_u8_setup, dim3(1), dim3(256), 0, s, hist, ctl, pk.hist_hi_dev, pk.hist_hi[0], pk.hist_hi[1]);
    hipError_t e = launch_pass1(img, n_px, w, pk, hist, ctl->range, nullptr, dev, s, h_out);
    if (e != hipSuccess || !pk.auto_range) return e;
    hipLaunchKernelGGL(k_range_check, dim3(1), dim3(256), 0, s, hist, ctl, pk.q64, range_out);
    return launch_pass1(img, n_px, w, pk, hist, ctl->range, &ctl->retry, dev, s);
}

hipError_t launch_densities(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                            float* h_out, uint64_t* hist, float* p99_out, int32_t* flags_out, float* range_out,
                            void* ctl_ws, const DevInfo& dev, hipStream_t s) {
    // the range check reports the settled range itself when the percentile is not asked for
    const bool range_only = pk.auto_range && range_out && !p99_out && !flags_out;
    hipError_t e = launch_hist_checked(img, n_px, w, pk, hist, ctl_ws, dev, s, h_out, range_only ? range_out : nullptr);
    if (e != hipSuccess) return e;
    if (!range_only && (p99_out || flags_out || range_out)) {
        U8Ctl* ctl = ctl_of(ctl_ws);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, hist, pk.q64, ctl->range, pk.hist_hi[0],
                           pk.hist_hi[1], &ctl->retry, w, pk.lambda, p99_out, flags_out, range_out);
    }
    return hipGetLastError();
}

static P2Args p2_args(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                      const float* scale_tgt, const float i0_out[3], const ParamsK& pk, uint8_t* out) {
    P2Args b{};
    b.src = src; b.out = out; b.n_px = n_px; b.w_src = w_src; b.w_tgt = w_tgt; b.scale_tgt = scale_tgt;
    for (int c = 0; c < 3; ++c) { b.i0[c] = pk.i0[c]; b.i0_out[c] = i0_out[c]; }
    b.lambda = pk.lambda; b.hist_hi[0] = pk.hist_hi[0]; b.hist_hi[1] = pk.hist_hi[1];
    b.range = pk.hist_hi_dev;
    b.q = pk.q64;
    return b;
}

static hipError_t run_recolor(const P2Args& b, const DevInfo& dev, hipStream_t s) {
    const int bpc = option(SPCN_OPT_P2_BLOCKS_PER_CU);
    switch (option(SPCN_OPT_P2_VARIANT)) {
        case 0: return run_pass2<1, 256>(b, bpc, dev, s);
        case 1: return run_pass2<4, 256>(b, bpc, dev, s);
        case 2: return run_pass2<16, 1024>(b, 1, dev, s);
        case 3: return run_pass2g<1, 256>(b, bpc, dev, s);
        case 4: return run_pass2g<1, 512>(b, bpc, dev, s);
        default: return run_pass2g<16, 1024>(b, 1, dev, s);
    }
}

hipError_t launch_recolor(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                          const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                          uint8_t* out, const uint64_t* hist, float* p99_out, float* scale_out,
                          int32_t* flags_out, float* range_out, const DevInfo& dev, hipStream_t s) {
    P2Args b = p2_args(src, n_px, w_src, w_tgt, scale_tgt, i0_out, pk, out);
    b.hist = hist;
    b.p99_out = p99_out; b.scale_out = scale_out; b.flags_out = flags_out; b.range_out = range_out;
    return run_recolor(b, dev, s);
}

hipError_t launch_recolor_p99(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                              const float* scale_tgt, const float i0_out[3], const ParamsK& pk, uint8_t* out,
                              const float* p99_in, float* scale_out, int32_t* flags_out, const DevInfo& dev,
                              hipStream_t s) {
    P2Args b = p2_args(src, n_px, w_src, w_tgt, scale_tgt, i0_out, pk, out);
    b.hist = nullptr; b.p99_in = p99_in;
    b.scale_out = scale_out; b.flags_out = flags_out;
    return run_recolor(b, dev, s);
}

hipError_t launch_normalize(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                            const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                            uint8_t* out, uint64_t* hist, void* ctl_ws, float* p99_out, float* scale_out,
                            int32_t* flags_out, float* range_out, const DevInfo& dev, hipStream_t s) {
    hipError_t e = launch_hist_checked(src, n_px, w_src, pk, hist, ctl_ws, dev, s);
    if (e != hipSuccess) return e;
    U8Ctl* ctl = ctl_of(ctl_ws);
    P2Args b = p2_args(src, n_px, w_src, w_tgt, scale_tgt, i0_out, pk, out);
    b.range = ctl->range; b.retry = &ctl->retry;
    b.hist = hist;
    b.p99_out = p99_out; b.scale_out = scale_out; b.flags_out = flags_out; b.range_out = range_out;
    return run_recolor(b, dev, s);
}

}  // namespace spcn
