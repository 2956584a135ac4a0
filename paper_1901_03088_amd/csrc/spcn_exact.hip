// spcn_exact.hip -- the exact order statistic of Eq. 3 over all non-white pixels of a uint8 image
// (Sec. 3.1 item 2: the percentile of the densities of the non-white pixels), without any
// histogram interpolation: per stain the k-th smallest FP64 density, k = max(1, ceil(q n)).
//
// A density depends on the pixel only through its colour, so the selection runs over colours:
//   1. pass 1 (the exact 2 x 256 histogram of spcn_densities) gives n and, per stain, the bin b
//      holding rank k and the rank r of the wanted value inside that bin;
//   2. k_exact_refine reads the image again and counts, per stain, the colours of the non-white
//      pixels whose density falls in bin b (the bin decided exactly as in pass 1, with its tables:
//      fixed-point sums, FP64 re-solve near an edge) into a table of 2^24 uint64 counts;
//   3. k_exact_compact turns the counted colours into a list of (FP64 density bits, count); a radix
//      selection over it (six digit passes: k_exact_digits builds the count-weighted digit histogram
//      of the entries that share the bits fixed so far, k_exact_pick fixes the next digit; the
//      table itself is scanned if the list overflowed) ends with the r-th smallest
//      density of the bin, which is the k-th smallest overall, since every pixel of a lower bin
//      has a smaller density and every pixel of a higher bin a larger one.
// Non-negative doubles order like their bit patterns, so the selection is exact; equal densities
// of different colours are one value.  Table and list cost 320 MiB of workspace, independent of
// the image size.
#include "spcn_internal.h"
#include "spcn_passes.hpp"

namespace spcn {

namespace {

constexpr int kColours = 1 << 24;
constexpr unsigned int kListCap = 1u << 21;   // (key, count) list per stain; beyond it the table is scanned
constexpr int kDigitBins = 2048;
constexpr int kPasses = 6;
// bits [shift, shift + width) of the key are fixed by each pass; bit 63 (sign) is always 0
__host__ __device__ constexpr int digit_shift(int pass) { return pass < 5 ? 52 - 11 * pass : 0; }
__host__ __device__ constexpr int digit_width(int pass) { return pass < 5 ? 11 : 8; }

constexpr int RF_THREADS = 1024;

struct ExactState {
    unsigned long long n;             // non-white pixels
    unsigned long long r[2];          // 1-based rank of the wanted value inside bin b (then inside the prefix)
    unsigned long long prefix[2];     // key bits fixed so far
    int kb[2];                        // bin b holding rank k; -1 without tissue
    int basis_ok;
    unsigned int n_list[2];           // counted colours of the bin (entries of the key list if <= kListCap)
    int pad;
};

struct ExactWs {
    uint64_t* hist;                   // [2][256]
    ExactState* st;
    unsigned long long* dhist;        // [2][2048]
    ulonglong2* list;                 // [2][kListCap] (FP64 key bits, count) of the counted colours
    unsigned long long* table;        // [2][2^24]
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

ExactWs carve(void* ws) {
    uint8_t* p = static_cast<uint8_t*>(ws);
    ExactWs w;
    w.hist = reinterpret_cast<uint64_t*>(p); p += a256(2 * kHistBins * sizeof(uint64_t));
    w.st = reinterpret_cast<ExactState*>(p); p += a256(sizeof(ExactState));
    w.dhist = reinterpret_cast<unsigned long long*>(p); p += a256(2 * kDigitBins * sizeof(unsigned long long));
    w.list = reinterpret_cast<ulonglong2*>(p); p += (size_t)2 * kListCap * sizeof(ulonglong2);
    w.table = reinterpret_cast<unsigned long long*>(p);
    return w;
}

// Inclusive prefix sum of one 64-bit value per thread over a 256-thread workgroup (wave scans, then
// the totals of the preceding waves); s_wsum holds 4 words.  Barriers inside.
__device__ inline unsigned long long scan256_u64(unsigned long long v, unsigned long long* s_wsum) {
    const int t = threadIdx.x, lane = t & 63;
    unsigned long long incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long up = __shfl_up(incl, o);
        if (lane >= o) incl += up;
    }
    if (lane == 63) s_wsum[t >> 6] = incl;
    __syncthreads();
    for (int w = 0; w < (t >> 6); ++w) incl += s_wsum[w];
    __syncthreads();
    return incl;
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

// Rank k of the order statistic, the bin holding it and the rank inside that bin (one workgroup of
// 256 threads, one bin per thread).
__global__ __launch_bounds__(256) void k_exact_rank(ExactWs w, double q, const float* wb, float lambda) {
    __shared__ unsigned long long s_wsum[4];
    __shared__ ExactState s;
    __shared__ unsigned long long s_n;
    const int t = threadIdx.x;
    if (t == 0) {
        Basis64 B;
        derive_basis(wb, lambda, B);
        s = ExactState{};
        s.basis_ok = B.ok;
        for (int j = 0; j < 2; ++j) { s.kb[j] = -1; s.r[j] = 0; s.prefix[j] = 0; }
    }
    const unsigned long long c0 = w.hist[t];
    const unsigned long long n_incl = scan256_u64(c0, s_wsum);
    if (t == 255) s_n = n_incl;
    __syncthreads();
    const unsigned long long n = s_n;
    if (t == 0) s.n = n;
    long long k = 0;
    if (n > 0) {
        k = (long long)ceil(q * (double)n);
        k = k < 1 ? 1 : (k > (long long)n ? (long long)n : k);
    }
    for (int j = 0; j < 2; ++j) {
        const unsigned long long c = j ? w.hist[kHistBins + t] : c0;
        const unsigned long long incl = scan256_u64(c, s_wsum);
        if (n > 0 && incl - c < (unsigned long long)k && (unsigned long long)k <= incl) {   // one thread
            s.kb[j] = t;
            s.r[j] = (unsigned long long)k - (incl - c);
        }
    }
    __syncthreads();
    if (t == 0) *w.st = s;
}

struct RefineArgs {
    const uint8_t* img;
    int64_t units;                    // full 4-pixel units
    int32_t tail;                     // pixels after them (0..3)
    const float* w;
    P1Params pp;
    ExactWs ws;
    int64_t scatter, step;            // tile permutation (see p1f_tiles)
};

__device__ __forceinline__ uint32_t colour_index(uint32_t R, uint32_t G, uint32_t B) { return R | (G << 8) | (B << 16); }

constexpr int RF_UNROLL = 2;

// Bin of a fixed-point sum of the byte-permute tables away from the bin edges (as pass 1 decides it).
template <bool U16>
__device__ __forceinline__ int refine_bin(int32_t y, int u) {
    return U16 ? (int)((uint32_t)min(max(y, 0), 0xFFFFFF) >> 16) : min(max(y >> u, 0), kHistBins - 1);
}

// One pixel known to be non-white and near an edge: FP64 bins, then the colour counts.
__device__ __forceinline__ void refine_exact(const P1FLds<true>& S, const P1Params& pp, uint32_t R, uint32_t G,
                                             uint32_t Bc, int kb0, int kb1, unsigned long long* t0,
                                             unsigned long long* t1) {
    double d0, d1;
    solve64(S.B, S.od[0][R], S.od[1][G], S.od[2][Bc], d0, d1);
    const double e0 = floor(d0 * (256.0 / (double)pp.hist_hi[0])), e1 = floor(d1 * (256.0 / (double)pp.hist_hi[1]));
    const int k0 = e0 >= 255.0 ? 255 : (int)e0, k1 = e1 >= 255.0 ? 255 : (int)e1;
    if (k0 == kb0) atomicAdd(t0 + colour_index(R, G, Bc), 1ull);
    if (k1 == kb1) atomicAdd(t1 + colour_index(R, G, Bc), 1ull);
}

// The pass-1 arithmetic of UNROLL units per thread (byte-permute tables, same near-edge rule), with
// the histogram add replaced by the colour count of the pixels in the selected bins.
template <bool U16>
__device__ __forceinline__ void refine_units(const P1FLds<true>& S, const P1Params& pp, const P1FLane& L,
                                             const u32x3 (&cur)[RF_UNROLL], int lb0, int cnt, int nthreads, int kb0,
                                             int kb1, unsigned long long* t0, unsigned long long* t1) {
    const int u = U16 ? 16 : S.shift;
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const uint32_t nmask = p1f_nmask(u);
    uint64_t near_waves = 0;
#pragma unroll
    for (int j = 0; j < RF_UNROLL; ++j) {
        const bool valid = lb0 + j * nthreads < cnt;
        const uint32_t X = cur[j].x, Y0 = cur[j].y, Z = cur[j].z;
        int32_t sum[4];
        sum[0] = (int32_t)__builtin_amdgcn_udot4(X, 0x00010101u, 0u, false);
        sum[1] = (int32_t)__builtin_amdgcn_udot4(Y0, 0x00000101u, __builtin_amdgcn_udot4(X, 0x01000000u, 0u, false), false);
        sum[2] = (int32_t)__builtin_amdgcn_udot4(Z, 0x00000001u, __builtin_amdgcn_udot4(Y0, 0x01010000u, 0u, false), false);
        sum[3] = (int32_t)__builtin_amdgcn_udot4(Z, 0x01010100u, 0u, false);
        const int32_t darkest = min(min(sum[0], sum[1]), min(sum[2], sum[3]));
        const uint64_t valid_lanes = __ballot(valid);
        if (valid && darkest < thr) {
            int32_t ys0[4], ys1[4];
            p1f_unit_sums(S, L, X, Y0, Z, ys0, ys1);
            // colour index (R | G << 8 | B << 16) of each pixel from the unit's dwords
            const uint32_t col[4] = {X & 0xFFFFFFu, __builtin_amdgcn_perm(Y0, X, 0x0c050403u),
                                     __builtin_amdgcn_perm(Z, Y0, 0x0c040302u), Z >> 8};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t y0 = ys0[q], y1 = ys1[q];
                const uint64_t white = __ballot(sum[q] >= thr);
                const uint64_t nr = __ballot(p1f_near(y0, nmask)) | __ballot(p1f_near(y1, nmask));
                near_waves |= nr & ~white & valid_lanes;
                if (__builtin_amdgcn_inverse_ballot_w64(valid_lanes & ~(white | nr))) {
                    if (refine_bin<U16>(y0, u) == kb0) atomicAdd(t0 + col[q], 1ull);
                    if (refine_bin<U16>(y1, u) == kb1) atomicAdd(t1 + col[q], 1ull);
                }
            }
        }
    }
    if (near_waves) {   // rare: the near-edge pixels of these units in FP64
#pragma unroll
        for (int j = 0; j < RF_UNROLL; ++j) {
            if (lb0 + j * nthreads >= cnt) continue;
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t R = px[q][0], G = px[q][1], Bc = px[q][2];
                if ((int32_t)(R + G + Bc) >= thr) continue;
                int32_t y0, y1;
                p1f_sums(S, R, G, Bc, L.r16, y0, y1);
                if (p1f_near(y0, nmask) | p1f_near(y1, nmask)) refine_exact(S, pp, R, G, Bc, kb0, kb1, t0, t1);
            }
        }
    }
}

// Counts, per stain, the colours of the non-white pixels whose density lies in the stain's bin b:
// grid-stride over scattered tiles as pass 1 (one 1024-thread workgroup per CU).
template <bool U16>
__device__ void refine_tiles(const P1FLds<true>& S, const RefineArgs& a, int kb0, int kb1) {
    const int tid = threadIdx.x;
    const P1FLane L = p1f_lane<true>(tid, a.pp.white_sum);
    const int64_t tu = (int64_t)RF_THREADS * RF_UNROLL;
    const int64_t n_tiles = (a.units + tu - 1) / tu;
    unsigned long long* t0 = a.ws.table;
    unsigned long long* t1 = a.ws.table + kColours;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    int64_t ph = (t * a.scatter) % n_tiles;
    auto tile_rs = [&](int64_t tt, int64_t tile) {
        const bool in = tt < n_tiles;
        return chunk_rsrc(a.img, in ? tile * tu : 0, in ? min(tu, a.units - tile * tu) : 0);
    };
    const __amdgpu_buffer_rsrc_t rs = tile_rs(t, ph);
    u32x3 cur[RF_UNROLL];
#pragma unroll
    for (int j = 0; j < RF_UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * RF_THREADS), 0, kLoadStream);
    for (; t < n_tiles; t += gridDim.x) {
        int64_t pn = ph + a.step;
        if (pn >= n_tiles) pn -= n_tiles;
        const __amdgpu_buffer_rsrc_t rn = tile_rs(t + gridDim.x, pn);
        u32x3 nxt[RF_UNROLL];
#pragma unroll
        for (int j = 0; j < RF_UNROLL; ++j) nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * RF_THREADS), 0, kLoadStream);
        const int cnt = (int)min(tu, a.units - ph * tu);
        refine_units<U16>(S, a.pp, L, cur, tid, cnt, RF_THREADS, kb0, kb1, t0, t1);
#pragma unroll
        for (int j = 0; j < RF_UNROLL; ++j) cur[j] = nxt[j];
        ph = pn;
    }
}

__global__ __launch_bounds__(RF_THREADS) void k_exact_refine(const RefineArgs a) {
    __shared__ P1FLds<true> S;
    p1f_setup(S, a.w, a.pp, false);
    const int kb0 = a.ws.st->kb[0], kb1 = a.ws.st->kb[1];
    if (kb0 < 0 && kb1 < 0) return;     // uniform over the grid: no tissue
    if (S.shift == 16) refine_tiles<true>(S, a, kb0, kb1);
    else refine_tiles<false>(S, a, kb0, kb1);
    if (blockIdx.x == 0 && threadIdx.x < a.tail) {
        const uint8_t* p = a.img + 12 * a.units + 3 * threadIdx.x;
        const uint32_t R = p[0], G = p[1], Bc = p[2];
        const int32_t thr = a.pp.white_sum > 0 ? a.pp.white_sum : 0x7FFFFFFF;
        if ((int32_t)(R + G + Bc) < thr)   // the tail in FP64 (at most 3 pixels)
            refine_exact(S, a.pp, R, G, Bc, kb0, kb1, a.ws.table, a.ws.table + kColours);
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
// FP64 density key of colour col for stain j (non-negative doubles order like their bit patterns).
__device__ __forceinline__ unsigned long long colour_key(const Basis64& B, const double (*od)[kHistBins], uint32_t col,
                                                         int j) {
    double d0, d1;
    solve64(B, od[0][col & 255], od[1][(col >> 8) & 255], od[2][col >> 16], d0, d1);
    const double d = j ? d1 : d0;
    return d > 0.0 ? (unsigned long long)__double_as_longlong(d) : 0ull;
}

// The counted colours of each stain as a list of (key, count), so that the digit passes read a few
// MB instead of the 256 MiB table (grid: x over colours, y = stain; appends aggregated per wave).
__global__ __launch_bounds__(256) void k_exact_compact(const DigitArgs a) {
    __shared__ double s_od[3][kHistBins];
    __shared__ Basis64 B;
    const int j = blockIdx.y;
    ExactState* st = a.ws.st;
    if (st->kb[j] < 0) return;                          // uniform per workgroup
    if (threadIdx.x == 0) derive_basis(a.w, a.lambda, B);
    for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
        for (int c = 0; c < 3; ++c) s_od[c][k] = od_u8((double)a.i0[c], k);
    __syncthreads();
    const ulonglong2* tab = reinterpret_cast<const ulonglong2*>(a.ws.table + (int64_t)j * kColours);
    ulonglong2* list = a.ws.list + (int64_t)j * kListCap;
    const int lane = threadIdx.x & 63;
    const int n2 = kColours / 2;                        // table pairs; the last stride is guarded
    for (int i0 = blockIdx.x * blockDim.x; i0 < n2; i0 += gridDim.x * blockDim.x) {   // uniform per wave
        const int i = i0 + threadIdx.x;
        const ulonglong2 c2 = i < n2 ? tab[i] : make_ulonglong2(0ull, 0ull);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned long long cnt = e ? c2.y : c2.x;
            const uint64_t m = __ballot(cnt != 0ull);
            if (!m) continue;                           // uniform
            unsigned int base = 0;
            if (lane == __ffsll((unsigned long long)m) - 1) base = atomicAdd(&st->n_list[j], (unsigned int)__popcll(m));
            base = __shfl(base, __ffsll((unsigned long long)m) - 1);
            if (cnt) {
                const unsigned int slot = base + (unsigned int)__popcll(m & ((1ull << lane) - 1ull));
                if (slot < kListCap) list[slot] = make_ulonglong2(colour_key(B, s_od, 2u * (uint32_t)i + e, j), cnt);
            }
        }
    }
}

// Count-weighted histogram of digit `pass` of the density keys of the counted colours whose key
// agrees with the stain's prefix on the bits above the digit (grid: x over entries, y = stain);
// from the list, or from the table when the list overflowed.
__global__ __launch_bounds__(256) void k_exact_digits(const DigitArgs a) {
    __shared__ double s_od[3][kHistBins];
    __shared__ Basis64 B;
    __shared__ unsigned long long s_h[kDigitBins];
    const int j = blockIdx.y;
    const ExactState* st = a.ws.st;
    if (st->kb[j] < 0) return;                          // uniform per workgroup
    const unsigned int n_list = st->n_list[j];
    const bool from_list = n_list <= kListCap;
    if (!from_list) {
        if (threadIdx.x == 0) derive_basis(a.w, a.lambda, B);
        for (int k = threadIdx.x; k < kHistBins; k += blockDim.x)
            for (int c = 0; c < 3; ++c) s_od[c][k] = od_u8((double)a.i0[c], k);
    }
    for (int i = threadIdx.x; i < kDigitBins; i += blockDim.x) s_h[i] = 0ull;
    __syncthreads();
    const int shift = digit_shift(a.pass), width = digit_width(a.pass);
    const int hi = shift + width;                       // <= 63
    const unsigned long long prefix = st->prefix[j];
    const unsigned long long dmask = (1ull << width) - 1;
    if (from_list) {
        const ulonglong2* list = a.ws.list + (int64_t)j * kListCap;
        for (unsigned int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_list; i += gridDim.x * blockDim.x) {
            const ulonglong2 kc = list[i];
            if (((kc.x ^ prefix) >> hi) == 0ull) atomicAdd(&s_h[(kc.x >> shift) & dmask], kc.y);
        }
    } else {
        const ulonglong2* tab = reinterpret_cast<const ulonglong2*>(a.ws.table + (int64_t)j * kColours);
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kColours / 2; i += gridDim.x * blockDim.x) {
            const ulonglong2 c2 = tab[i];
            if ((c2.x | c2.y) == 0ull) continue;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const unsigned long long cnt = e ? c2.y : c2.x;
                if (!cnt) continue;
                const unsigned long long key = colour_key(B, s_od, 2u * (uint32_t)i + (uint32_t)e, j);
                if (((key ^ prefix) >> hi) == 0ull) atomicAdd(&s_h[(key >> shift) & dmask], cnt);
            }
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
    __shared__ unsigned long long s_wsum[4];
    __shared__ int s_g;
    __shared__ unsigned long long s_below;
    const int j = blockIdx.x, t = threadIdx.x;
    ExactState* st = w.st;
    const bool live = st->kb[j] >= 0;                   // uniform per workgroup
    constexpr int per = kDigitBins / 256;
    unsigned long long* dh = w.dhist + j * kDigitBins;
    if (live) {
        const unsigned long long r = st->r[j];
        unsigned long long sum = 0;
#pragma unroll
        for (int i = 0; i < per; ++i) sum += dh[t * per + i];
        const unsigned long long incl = scan256_u64(sum, s_wsum);
        if (t == 255) { s_g = 255; s_below = incl - sum; }   // default if the counts fall short of r
        __syncthreads();
        if (incl - sum < r && r <= incl) { s_g = t; s_below = incl - sum; }   // at most one thread
        __syncthreads();
        if (t < 64) {   // the group's digits, one lane each
            const int g = s_g;
            const unsigned long long c = t < per ? dh[g * per + t] : 0ull;
            unsigned long long in = c;
            for (int o = 1; o < per; o <<= 1) {
                const unsigned long long up = __shfl_up(in, o);
                if (t >= o) in += up;
            }
            const unsigned long long rr = r - s_below;
            const uint64_t m = __ballot(t < per && in - c < rr && rr <= in);
            const int who = m ? __ffsll((unsigned long long)m) - 1 : per - 1;
            const unsigned long long before = __shfl(in - c, who);
            if (t == 0) {
                st->r[j] = rr - before;
                st->prefix[j] |= (unsigned long long)(g * per + who) << digit_shift(pass);
            }
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
           a256(2 * kDigitBins * sizeof(unsigned long long)) + (size_t)2 * kListCap * sizeof(ulonglong2) +
           (size_t)2 * kColours * sizeof(unsigned long long);
}

hipError_t launch_exact_percentile(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk_in,
                                   float* p99_out, int32_t* flags_out, void* ws, const DevInfo& dev, hipStream_t s) {
    ParamsK pk = pk_in;
    pk.hist_hi_dev = nullptr;   // the range only places the bins of the first read: the host value serves
    ExactWs x = carve(ws);
    hipError_t e = launch_zero_hist(x.hist, s);
    if (e != hipSuccess) return e;
    if ((e = launch_count(img, n_px, w, pk, x.hist, dev, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_clear, dim3((unsigned)dev.cus * 8), dim3(256), 0, s, x);
    hipLaunchKernelGGL(k_exact_rank, dim3(1), dim3(256), 0, s, x, pk.q64, w, pk.lambda);
    RefineArgs ra{};
    ra.img = img; ra.units = n_px / 4; ra.tail = (int32_t)(n_px % 4); ra.w = w;
    for (int c = 0; c < 3; ++c) ra.pp.i0[c] = pk.i0[c];
    ra.pp.lambda = pk.lambda; ra.pp.white_sum = pk.white_sum;
    ra.pp.hist_hi[0] = pk.hist_hi[0]; ra.pp.hist_hi[1] = pk.hist_hi[1];
    ra.ws = x;
    const int64_t rf_tiles = (ra.units + (int64_t)RF_THREADS * RF_UNROLL - 1) / ((int64_t)RF_THREADS * RF_UNROLL);
    const int64_t grid = rf_tiles < (int64_t)dev.cus ? (rf_tiles > 0 ? rf_tiles : 1) : (int64_t)dev.cus;
    ra.scatter = tile_scatter(rf_tiles, grid);
    ra.step = rf_tiles > 0 ? (grid * ra.scatter) % rf_tiles : 0;
    hipLaunchKernelGGL(k_exact_refine, dim3((unsigned)grid), dim3(RF_THREADS), 0, s, ra);
    DigitArgs da{};
    da.ws = x; da.w = w; da.lambda = pk.lambda;
    for (int c = 0; c < 3; ++c) da.i0[c] = pk.i0[c];
    hipLaunchKernelGGL(k_exact_compact, dim3((unsigned)dev.cus * 4, 2), dim3(256), 0, s, da);
    for (int pass = 0; pass < kPasses; ++pass) {
        da.pass = pass;
        hipLaunchKernelGGL(k_exact_digits, dim3((unsigned)dev.cus * 2, 2), dim3(256), 0, s, da);
        hipLaunchKernelGGL(k_exact_pick, dim3(2), dim3(256), 0, s, x, pass, p99_out, flags_out);
    }
    return hipGetLastError();
}

}  // namespace spcn
