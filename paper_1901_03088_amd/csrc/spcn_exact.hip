// spcn_exact.hip -- the exact order statistic of Eq. 3 over all non-white pixels of a uint8 image
// (Sec. 3.1 item 2: the percentile of the densities of the non-white pixels), without any
// histogram interpolation: per stain the k-th smallest FP64 density, k = max(1, ceil(q n)).
//
// A density depends on the pixel only through its colour, so the selection runs over colours:
//   1. pass 1 (the exact 2 x 256 histogram of spcn_densities) gives n and, per stain, the bin b
//      holding rank k and the rank r of the wanted value inside that bin;
//   2. k_exact_refine reads the image again and counts, per stain, the colours of the non-white
//      pixels whose density falls in bin b (the bin decided exactly as in pass 1: fixed-point
//      tables, FP64 re-solve near an edge) into a table of 2^24 uint64 counts;
//   3. a radix selection over the FP64 bit patterns of the densities of the counted colours (six
//      digit passes: k_exact_digits builds the count-weighted digit histogram of the colours that
//      share the bits fixed so far, k_exact_pick fixes the next digit) ends with the r-th smallest
//      density of the bin, which is the k-th smallest overall, since every pixel of a lower bin
//      has a smaller density and every pixel of a higher bin a larger one.
// Non-negative doubles order like their bit patterns, so the selection is exact; equal densities
// of different colours are one value.  The table costs 256 MiB of workspace, independent of the
// image size.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int kColours = 1 << 24;
constexpr int kDigitBins = 2048;
constexpr int kPasses = 6;
// bits [shift, shift + width) of the key are fixed by each pass; bit 63 (sign) is always 0
__host__ __device__ constexpr int digit_shift(int pass) { return pass < 5 ? 52 - 11 * pass : 0; }
__host__ __device__ constexpr int digit_width(int pass) { return pass < 5 ? 11 : 8; }

constexpr int RF_THREADS = 1024;
constexpr int RF_CHUNK = 16384;          // 4-pixel units per workgroup iteration

struct ExactState {
    unsigned long long n;             // non-white pixels
    unsigned long long r[2];          // 1-based rank of the wanted value inside bin b (then inside the prefix)
    unsigned long long prefix[2];     // key bits fixed so far
    int kb[2];                        // bin b holding rank k; -1 without tissue
    int basis_ok;
    int pad;
};

struct ExactWs {
    uint64_t* hist;                   // [2][256]
    ExactState* st;
    unsigned long long* dhist;        // [2][2048]
    unsigned long long* table;        // [2][2^24]
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

ExactWs carve(void* ws) {
    uint8_t* p = static_cast<uint8_t*>(ws);
    ExactWs w;
    w.hist = reinterpret_cast<uint64_t*>(p); p += a256(2 * kHistBins * sizeof(uint64_t));
    w.st = reinterpret_cast<ExactState*>(p); p += a256(sizeof(ExactState));
    w.dhist = reinterpret_cast<unsigned long long*>(p); p += a256(2 * kDigitBins * sizeof(unsigned long long));
    w.table = reinterpret_cast<unsigned long long*>(p);
    return w;
}

// Fill kernel (capturable): the colour table and the digit histograms.
__global__ __launch_bounds__(256) void k_exact_clear(ExactWs w) {
    const int64_t n4 = (int64_t)2 * kColours / 2;      // ulonglong2 stores
    ulonglong2* t = reinterpret_cast<ulonglong2*>(w.table);
    const ulonglong2 z = {0ull, 0ull};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        t[i] = z;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 2 * kDigitBins; i += blockDim.x) w.dhist[i] = 0ull;
}

// Rank k of the order statistic, the bin holding it and the rank inside that bin (one wavefront).
__global__ __launch_bounds__(64) void k_exact_rank(ExactWs w, double q, const float* wb, float lambda) {
    if (threadIdx.x != 0) return;
    Basis64 B;
    derive_basis(wb, lambda, B);
    ExactState s{};
    unsigned long long n = 0;
    for (int b = 0; b < kHistBins; ++b) n += w.hist[b];
    s.n = n;
    s.basis_ok = B.ok;
    for (int j = 0; j < 2; ++j) {
        s.kb[j] = -1;
        s.r[j] = 0;
        s.prefix[j] = 0;
        if (n == 0) continue;
        long long k = (long long)ceil(q * (double)n);
        k = k < 1 ? 1 : (k > (long long)n ? (long long)n : k);
        unsigned long long below = 0;
        int b = 0;
        const uint64_t* h = w.hist + j * kHistBins;
        while (b < kHistBins - 1 && below + h[b] < (unsigned long long)k) below += h[b++];
        s.kb[j] = b;
        s.r[j] = (unsigned long long)k - below;
    }
    *w.st = s;
}

struct RefineArgs {
    const uint8_t* img;
    int64_t units;                    // full 4-pixel units
    int32_t tail;                     // pixels after them (0..3)
    const float* w;
    P1Params pp;
    ExactWs ws;
};

__device__ __forceinline__ uint32_t colour_index(uint32_t R, uint32_t G, uint32_t B) { return R | (G << 8) | (B << 16); }

// Counts, per stain, the colours of the non-white pixels whose density lies in the stain's bin b.
__global__ __launch_bounds__(RF_THREADS) void k_exact_refine(const RefineArgs a) {
    using L = P1Lds<4, 1>;
    __shared__ L S;
    p1_setup(S, a.w, a.pp, false);
    const int kb0 = a.ws.st->kb[0], kb1 = a.ws.st->kb[1];
    if (kb0 < 0 && kb1 < 0) return;     // uniform over the grid: no tissue
    const int tid = threadIdx.x;
    const int u = S.shift;
    const int32_t thr = a.pp.white_sum > 0 ? a.pp.white_sum : 0x7FFFFFFF;
    const int32_t fmask = (1 << u) - 1;
    const uint32_t roff = (uint32_t)(tid & 3) << 4;
    const char* tb = reinterpret_cast<const char*>(S.tab);
    const double sg0 = 256.0 / (double)a.pp.hist_hi[0], sg1 = 256.0 / (double)a.pp.hist_hi[1];
    unsigned long long* t0 = a.ws.table;
    unsigned long long* t1 = a.ws.table + kColours;

    auto pixel = [&](uint32_t R, uint32_t G, uint32_t Bc, bool valid) {
        if (!valid || (int32_t)(R + G + Bc) >= thr) return;
        const int4 e0 = *reinterpret_cast<const int4*>(tb + ((R << L::kShift) | roff));
        const int4 e1 = *reinterpret_cast<const int4*>(tb + L::kChannelBytes + ((G << L::kShift) | roff));
        const int4 e2 = *reinterpret_cast<const int4*>(tb + 2 * L::kChannelBytes + ((Bc << L::kShift) | roff));
        const int32_t x0 = min(e0.x + e1.x + e2.x, e0.y + e1.y + e2.y);
        const int32_t x1 = min(e0.z + e1.z + e2.z, e0.w + e1.w + e2.w);
        int k0 = min(max(x0 >> u, 0), kHistBins - 1);
        int k1 = min(max(x1 >> u, 0), kHistBins - 1);
        if (near_edge(x0, fmask) | near_edge(x1, fmask)) {
            double d0, d1;
            solve64(S.B, od_u8((double)a.pp.i0[0], (int)R), od_u8((double)a.pp.i0[1], (int)G),
                    od_u8((double)a.pp.i0[2], (int)Bc), d0, d1);
            const double f0 = floor(d0 * sg0), f1 = floor(d1 * sg1);
            k0 = f0 >= 255.0 ? 255 : (int)f0;
            k1 = f1 >= 255.0 ? 255 : (int)f1;
        }
        if (k0 == kb0) atomicAdd(t0 + colour_index(R, G, Bc), 1ull);
        if (k1 == kb1) atomicAdd(t1 + colour_index(R, G, Bc), 1ull);
    };

    const int64_t n_chunks = (a.units + RF_CHUNK - 1) / RF_CHUNK;
    for (int64_t c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const int64_t u0 = c * RF_CHUNK;
        const int cnt = (int)min((int64_t)RF_CHUNK, a.units - u0);
        const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.img, u0, cnt);
        for (int lb = tid; lb < cnt; lb += RF_THREADS) {
            const u32x3 d = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * lb, 0, 0);
            uint32_t px[4][3];
            bytes_of_unit(d, px);
#pragma unroll
            for (int q = 0; q < 4; ++q) pixel(px[q][0], px[q][1], px[q][2], true);
        }
    }
    if (blockIdx.x == 0 && tid < a.tail) {
        const uint8_t* p = a.img + 12 * a.units + 3 * tid;
        pixel(p[0], p[1], p[2], true);
    }
}

struct DigitArgs {
    ExactWs ws;
    const float* w;
    float lambda;
    float i0[3];
    int pass;
};

// Count-weighted histogram of digit `pass` of the density keys of the counted colours whose key
// agrees with the stain's prefix on the bits above the digit (grid: x over colours, y = stain).
__global__ __launch_bounds__(256) void k_exact_digits(const DigitArgs a) {
    __shared__ double s_od[3][kHistBins];
    __shared__ Basis64 B;
    __shared__ unsigned long long s_h[kDigitBins];
    const int j = blockIdx.y;
    const ExactState* st = a.ws.st;
    if (st->kb[j] < 0) return;                          // uniform per workgroup
    if (threadIdx.x == 0) derive_basis(a.w, a.lambda, B);
    for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
        for (int c = 0; c < 3; ++c) s_od[c][k] = od_u8((double)a.i0[c], k);
    for (int i = threadIdx.x; i < kDigitBins; i += blockDim.x) s_h[i] = 0ull;
    __syncthreads();
    const int shift = digit_shift(a.pass), width = digit_width(a.pass);
    const int hi = shift + width;                       // <= 63
    const unsigned long long prefix = st->prefix[j];
    const unsigned long long dmask = (1ull << width) - 1;
    const ulonglong2* tab = reinterpret_cast<const ulonglong2*>(a.ws.table + (int64_t)j * kColours);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kColours / 2; i += gridDim.x * blockDim.x) {
        const ulonglong2 c2 = tab[i];
        if ((c2.x | c2.y) == 0ull) continue;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned long long cnt = e ? c2.y : c2.x;
            if (!cnt) continue;
            const uint32_t col = 2u * (uint32_t)i + (uint32_t)e;
            double d0, d1;
            solve64(B, s_od[0][col & 255], s_od[1][(col >> 8) & 255], s_od[2][col >> 16], d0, d1);
            const double d = j ? d1 : d0;
            const unsigned long long key = d > 0.0 ? (unsigned long long)__double_as_longlong(d) : 0ull;
            if (((key ^ prefix) >> hi) == 0ull) atomicAdd(&s_h[(key >> shift) & dmask], cnt);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kDigitBins; i += blockDim.x)
        if (s_h[i]) atomicAdd(a.ws.dhist + j * kDigitBins + i, s_h[i]);
}

// Fixes digit `pass` of stain blockIdx.x: the smallest digit whose cumulative count reaches the
// remaining rank; clears the digit histogram for the next pass; after the last pass writes the
// value and the flags.
__global__ __launch_bounds__(256) void k_exact_pick(ExactWs w, int pass, float* p99_out, int32_t* flags_out) {
    __shared__ unsigned long long s_part[256];
    __shared__ int s_g;
    const int j = blockIdx.x, t = threadIdx.x;
    ExactState* st = w.st;
    const bool live = st->kb[j] >= 0;
    constexpr int per = kDigitBins / 256;
    unsigned long long* dh = w.dhist + j * kDigitBins;
    if (live) {
        unsigned long long sum = 0;
        for (int i = 0; i < per; ++i) sum += dh[t * per + i];
        s_part[t] = sum;
        __syncthreads();
        if (t == 0) {
            unsigned long long r = st->r[j], below = 0;
            int g = 0;
            while (g < 255 && below + s_part[g] < r) { below += s_part[g]; ++g; }
            int d = g * per;
            while (d < g * per + per - 1 && below + dh[d] < r) { below += dh[d]; ++d; }
            st->r[j] = r - below;
            st->prefix[j] |= (unsigned long long)d << digit_shift(pass);
            s_g = g;
        }
        __syncthreads();
        for (int i = t; i < kDigitBins; i += blockDim.x) dh[i] = 0ull;
    }
    if (pass == kPasses - 1 && t == 0) {
        const double P = live ? __longlong_as_double((long long)st->prefix[j]) : 0.0;
        p99_out[j] = (float)P;
        if (flags_out)
            flags_out[j] = (live ? 0 : SPCN_FLAG_NO_TISSUE) | (st->basis_ok ? 0 : SPCN_FLAG_BASIS);
    }
}

}  // namespace

size_t exact_workspace_bytes() {
    return a256(2 * kHistBins * sizeof(uint64_t)) + a256(sizeof(ExactState)) +
           a256(2 * kDigitBins * sizeof(unsigned long long)) + (size_t)2 * kColours * sizeof(unsigned long long);
}

hipError_t launch_exact_percentile(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                                   float* p99_out, int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s) {
    ExactWs x = carve(ws);
    hipError_t e = launch_zero_hist(x.hist, s);
    if (e != hipSuccess) return e;
    if ((e = launch_count(img, n_px, w, pk, x.hist, dev, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_clear, dim3((unsigned)dev.cus * 8), dim3(256), 0, s, x);
    hipLaunchKernelGGL(k_exact_rank, dim3(1), dim3(64), 0, s, x, pk.q64, w, pk.lambda);
    RefineArgs ra{};
    ra.img = img; ra.units = n_px / 4; ra.tail = (int32_t)(n_px % 4); ra.w = w;
    for (int c = 0; c < 3; ++c) ra.pp.i0[c] = pk.i0[c];
    ra.pp.lambda = pk.lambda; ra.pp.white_sum = pk.white_sum;
    ra.pp.hist_hi[0] = pk.hist_hi[0]; ra.pp.hist_hi[1] = pk.hist_hi[1];
    ra.ws = x;
    const int64_t n_chunks = (ra.units + RF_CHUNK - 1) / RF_CHUNK;
    const int64_t grid = n_chunks < (int64_t)dev.cus * 2 ? (n_chunks > 0 ? n_chunks : 1) : (int64_t)dev.cus * 2;
    hipLaunchKernelGGL(k_exact_refine, dim3((unsigned)grid), dim3(RF_THREADS), 0, s, ra);
    DigitArgs da{};
    da.ws = x; da.w = w; da.lambda = pk.lambda;
    for (int c = 0; c < 3; ++c) da.i0[c] = pk.i0[c];
    for (int pass = 0; pass < kPasses; ++pass) {
        da.pass = pass;
        hipLaunchKernelGGL(k_exact_digits, dim3((unsigned)dev.cus * 2, 2), dim3(256), 0, s, da);
        hipLaunchKernelGGL(k_exact_pick, dim3(2), dim3(256), 0, s, x, pass, p99_out, flags_out);
    }
    return hipGetLastError();
}

}  // namespace spcn
