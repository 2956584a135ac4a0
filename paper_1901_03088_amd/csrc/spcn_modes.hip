// spcn_modes.hip -- the paper's median of per-patch percentiles (Sec. 3.2 items 3-4) on gfx950.
//
// Patches are bands of band_rows full rows (the paper's longitudinal patches).  Each band gets its
// own exact 2 x 256 non-white histogram from the pass-1 machinery (same tables, same exactness),
// its own histogram percentile (the formula of the global one, Eq. 3), and the median over the
// bands that hold non-white pixels is taken in FP64: the middle value, or the mean of the two
// middle values for an even count.
//
//   k_band_zero    clears the per-band histograms (a fill kernel: capturable);
//   k_band_hist    grid of (band, part) workgroups; each counts a contiguous part of its band's
//                  aligned 4-pixel units, the band's first workgroup also its unaligned head/tail;
//   k_band_final   one workgroup per band: percentile and flags;
//   k_band_median  one workgroup: rank selection of the middle band percentile(s) per stain.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int BH_THREADS = 1024;
constexpr int BH_UNROLL = 2;

int64_t hmin(int64_t a, int64_t b) { return a < b ? a : b; }
int64_t hmax(int64_t a, int64_t b) { return a > b ? a : b; }

struct BandArgs {
    const uint8_t* img;
    int64_t height, width, band_rows;
    int32_t n_bands, parts;          // workgroups per band
    const float* w;
    P1Params pp;
    unsigned long long* hist;        // [n_bands][2][256]
};

__global__ void k_band_zero(unsigned long long* h, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        h[i] = 0ull;
}

__global__ __launch_bounds__(BH_THREADS, 4) void k_band_hist(const BandArgs a) {
    __shared__ P1FLds<true> S;
    const P1Params pp = p1_resolve(a.pp);
    p1f_setup(S, a.w, pp, true);
    const int band = blockIdx.x / a.parts, part = blockIdx.x % a.parts;
    const int64_t r0 = (int64_t)band * a.band_rows;
    const int64_t r1 = min(a.height, r0 + a.band_rows);
    const int64_t p0 = r0 * a.width, p1 = r1 * a.width;
    const int64_t a0 = (p0 + 3) & ~(int64_t)3, a1 = p1 & ~(int64_t)3;   // aligned unit range
    const int64_t units = a1 > a0 ? (a1 - a0) >> 2 : 0;
    const int64_t per = (units + a.parts - 1) / a.parts;
    const int64_t u0 = min(units, (int64_t)part * per);
    const int cnt = (int)(min(units, u0 + per) - u0);
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.img + 3 * a0, u0, cnt);
    if (S.shift == 16)
        p1f_run<true, BH_UNROLL, true>(S, pp, rs, cnt, threadIdx.x, BH_THREADS);
    else
        p1f_run<true, BH_UNROLL, false>(S, pp, rs, cnt, threadIdx.x, BH_THREADS);
    if (part == 0 && threadIdx.x == 0) {
        if (a1 > a0) {
            p1f_tail(S, pp, a.img + 3 * p0, (int)(a0 - p0));
            p1f_tail(S, pp, a.img + 3 * a1, (int)(p1 - a1));
        } else {
            p1f_tail(S, pp, a.img + 3 * p0, (int)(p1 - p0));   // a band of fewer than 8 pixels
        }
    }
    p1f_merge(S, a.hist + (int64_t)band * 2 * kHistBins);
}

__global__ __launch_bounds__(256) void k_band_final(const uint64_t* hist, double q, const float* range, float hh0,
                                                    float hh1, const float* w, float lambda, double* band_P,
                                                    int32_t* band_F, float* band_out) {
    __shared__ FinalShared F;
    __shared__ int basis_ok;
    const float hh[2] = {resolve_range(range, hh0), resolve_range(range ? range + 1 : nullptr, hh1)};
    const int b = blockIdx.x;
    if (threadIdx.x == 0) { Basis64 B; derive_basis(w, lambda, B); basis_ok = B.ok; }
    block_percentiles(hist + (int64_t)b * 2 * kHistBins, q, hh, F);
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        band_P[2 * b + j] = F.P[j];
        band_F[2 * b + j] = stain_flags(F, j, basis_ok);
        if (band_out) band_out[2 * b + j] = (float)F.P[j];
    }
}

// Median over bands with non-white pixels: the element of rank m/2 (and m/2 - 1 for even m) in the
// order (value, band index).
__global__ __launch_bounds__(1024) void k_band_median(const double* band_P, const int32_t* band_F, int n_bands,
                                                      float* median_out, int32_t* flags_out) {
    __shared__ double s_pick[2][2];
    __shared__ int s_m[2];
    for (int j = 0; j < 2; ++j) {
        if (threadIdx.x == 0) s_m[j] = 0;
        __syncthreads();
        int cnt = 0;
        for (int b = threadIdx.x; b < n_bands; b += blockDim.x) cnt += !(band_F[2 * b + j] & SPCN_FLAG_NO_TISSUE);
        atomicAdd(&s_m[j], cnt);
        __syncthreads();
        const int m = s_m[j];
        for (int b = threadIdx.x; b < n_bands; b += blockDim.x) {
            if (band_F[2 * b + j] & SPCN_FLAG_NO_TISSUE) continue;
            const double v = band_P[2 * b + j];
            int rank = 0;
            for (int c = 0; c < n_bands; ++c) {
                if (band_F[2 * c + j] & SPCN_FLAG_NO_TISSUE) continue;
                const double u = band_P[2 * c + j];
                rank += (u < v) || (u == v && c < b);
            }
            if (rank == m / 2) s_pick[j][1] = v;
            if ((m & 1) == 0 && rank == m / 2 - 1) s_pick[j][0] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double med = 0.0;
            if (m > 0) med = (m & 1) ? s_pick[j][1] : 0.5 * (s_pick[j][0] + s_pick[j][1]);
            median_out[j] = (float)med;
            if (flags_out) flags_out[j] = m == 0 ? SPCN_FLAG_NO_TISSUE : 0;
        }
        __syncthreads();
    }
}

}  // namespace

size_t band_workspace_bytes(int64_t n_bands) {
    if (n_bands <= 0) return 0;
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return a256((size_t)n_bands * 2 * kHistBins * sizeof(uint64_t)) + a256((size_t)n_bands * 2 * sizeof(double)) +
           a256((size_t)n_bands * 2 * sizeof(int32_t));
}

hipError_t launch_band_percentiles(const uint8_t* img, int64_t height, int64_t width, const float* w,
                                   const ParamsK& pk, int64_t band_rows, float* band_out, float* median_out,
                                   int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s) {
    const int n_bands = (int)((height + band_rows - 1) / band_rows);
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    uint8_t* p = static_cast<uint8_t*>(ws);
    unsigned long long* hist = reinterpret_cast<unsigned long long*>(p);
    p += a256((size_t)n_bands * 2 * kHistBins * sizeof(uint64_t));
    double* band_P = reinterpret_cast<double*>(p); p += a256((size_t)n_bands * 2 * sizeof(double));
    int32_t* band_F = reinterpret_cast<int32_t*>(p);
    const int64_t nh = (int64_t)n_bands * 2 * kHistBins;
    hipLaunchKernelGGL(k_band_zero, dim3((unsigned)hmin((nh + 255) / 256, (int64_t)1024)), dim3(256), 0, s, hist, nh);
    BandArgs a{};
    a.img = img; a.height = height; a.width = width; a.band_rows = band_rows; a.n_bands = n_bands;
    // about four workgroups per CU in total (they run one per CU at a time, so the hardware balances
    // bands of unequal tissue content), at least one per band, parts of at least 64k units
    const int64_t band_units = band_rows * width / 4;
    int64_t parts = (4 * (int64_t)dev.cus + n_bands - 1) / n_bands;
    parts = hmin(parts, hmax((int64_t)1, band_units / 65536));
    parts = hmax(parts, (band_units + (1 << 26) - 1) >> 26);   // a part's bytes stay below 2^32
    a.parts = (int32_t)hmax((int64_t)1, parts);
    a.w = w;
    for (int c = 0; c < 3; ++c) a.pp.i0[c] = pk.i0[c];
    a.pp.lambda = pk.lambda; a.pp.white_sum = pk.white_sum;
    a.pp.hist_hi[0] = pk.hist_hi[0]; a.pp.hist_hi[1] = pk.hist_hi[1];
    a.pp.range = pk.hist_hi_dev;
    a.hist = hist;
    hipLaunchKernelGGL(k_band_hist, dim3((unsigned)(n_bands * a.parts)), dim3(BH_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_band_final, dim3((unsigned)n_bands), dim3(256), 0, s, (const uint64_t*)hist, pk.q64,
                       pk.hist_hi_dev, pk.hist_hi[0], pk.hist_hi[1], w, pk.lambda, band_P, band_F, band_out);
    hipLaunchKernelGGL(k_band_median, dim3(1), dim3(1024), 0, s, (const double*)band_P, (const int32_t*)band_F, n_bands,
                       median_out, flags_out);
    return hipGetLastError();
}

}  // namespace spcn
