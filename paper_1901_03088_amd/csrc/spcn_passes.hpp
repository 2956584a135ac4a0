// spcn_passes.hpp -- the two streaming passes of SPCN as workgroup-level building blocks, shared by
// the single-image kernels (spcn_u8.hip) and the persistent batched kernel (spcn_batched.hip).
//
//   pass 1: Eq. 1 + Eq. 2 per non-white pixel (Sec. 3.1 item 2) and an exact 2 x 256-bin histogram
//           of the two densities (the order statistic of Eq. 3 is taken from it);
//   pass 2: Eq. 1 + Eq. 2 again, the scaled recolouring of Eq. 3 and Eq. 4, written as uint8.
//
// Pixels travel as 4-pixel units (12 bytes, one buffer_load_dwordx3 per lane): a wavefront moves
// 768 contiguous bytes per instruction.  A chunk of units is addressed through a buffer resource
// with 32-bit offsets; the hardware range check returns zeros past the chunk (loads) and drops
// writes past it (stores).  Loads for the next iteration are issued before the current one is
// processed.
//
// Pass-1 tables: the candidates p_j and f_j of each stain (see spcn_device.hpp) are affine in the
// optical densities, so each is a sum of three per-channel int32 entries in 2^-u bin units; integer
// sums are exact, every entry is within 1/2 unit of its FP64 value, and a pixel whose value lies
// within kGuardUnits of a bin edge is re-solved in FP64 before it is counted.  Each 16-byte entry is
// replicated COPIES times and interleaved (entry k, copy r at (k * COPIES + r) * 16 bytes); lane l
// reads copy l % COPIES.  gfx950 serves 16-byte LDS reads 16 lanes per cycle (64 banks), so with
// fewer than 16 copies lanes l and l + COPIES of a cycle meet in the same banks unless they read the
// same entry.  The histogram keeps one private column per lane % COLS; LDS atomics are served 16 lanes
// per cycle, so 16 columns keep the lanes of a cycle in distinct banks.
#pragma once

#include "spcn_device.hpp"
#include "../../include/spcn.h"

#include <cstddef>

namespace spcn {

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufDword3 = 0x00020000;   // raw (untyped) buffer, gfx9-family descriptor word 3
// Cache policy of the streaming accesses (the cache-policy operand of the buffer instructions).
// Each pass reads the image once and writes its output once, so loads are non-temporal (nt) and
// stores non-temporal at device scope (sc1 nt): on a 6 GB buffer this takes a read-only sweep from
// 0.96 to 0.86 ms and a copy from 2.29 to 2.14 ms against the default policy.
constexpr int kLoadStream = 2;
constexpr int kStoreStream = 18;

// Buffer resource over `units` 12-byte units starting at unit `unit0` of `base`.  Every argument
// must be the same in all lanes of the wavefront (a workgroup's chunk): the fields are moved to
// scalar registers explicitly, because a descriptor the compiler keeps in vector registers is
// wrapped in a per-access loop over distinct lane values.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void* base, int64_t unit0, int64_t units) {
    const uint64_t addr = reinterpret_cast<uint64_t>(base) + 12 * (uint64_t)unit0;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)(12 * units));
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, n, kBufDword3);
}

__device__ __forceinline__ void bytes_of_unit(u32x3 d, uint32_t px[4][3]) {
    px[0][0] = d.x & 0xFF;         px[0][1] = (d.x >> 8) & 0xFF;  px[0][2] = (d.x >> 16) & 0xFF;
    px[1][0] = d.x >> 24;          px[1][1] = d.y & 0xFF;         px[1][2] = (d.y >> 8) & 0xFF;
    px[2][0] = (d.y >> 16) & 0xFF; px[2][1] = d.y >> 24;          px[2][2] = d.z & 0xFF;
    px[3][0] = (d.z >> 8) & 0xFF;  px[3][1] = (d.z >> 16) & 0xFF; px[3][2] = d.z >> 24;
}

// ================================================================================== pass 1

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }

template <int COPIES, int COLS>
struct P1Lds {
    static_assert((COPIES & (COPIES - 1)) == 0 && (COLS & (COLS - 1)) == 0, "powers of two");
    static constexpr int kChannelBytes = kHistBins * COPIES * 16;
    static constexpr int kShift = ilog2(COPIES * 16);
    int4 tab[3 * kHistBins * COPIES];          // (p0, f0, p1, f1) + guard offset, fixed point
    uint32_t hist[2 * kHistBins * COLS];       // [stain][bin][column]
    Basis64 B;
    int shift;
};

struct P1Params {
    float i0[3];
    float lambda;
    int32_t white_sum;
    float hist_hi[2];
    const float* range;     // device [2] range that replaces hist_hi when non-NULL (see resolve_range)
};

// The parameters with the histogram range settled (every kernel calls this once at its start).
__device__ inline P1Params p1_resolve(const P1Params& in) {
    P1Params p = in;
    p.hist_hi[0] = resolve_range(in.range, in.hist_hi[0]);
    p.hist_hi[1] = resolve_range(in.range ? in.range + 1 : nullptr, in.hist_hi[1]);
    p.range = nullptr;
    return p;
}

// A fixed-point sum x (value + guard, in units of 2^-u bin) decides its bin only if it is not within
// the guard band of an edge k * 2^u with k >= 1.  Edge 0 needs no decision: every value below
// 2^u, negative ones included (h = max(0, .)), lands in bin 0.
__device__ __forceinline__ bool near_edge(int32_t x, int32_t fmask) {
    return ((x & fmask) < 2 * kGuardUnits) & (x >= 2 * kGuardUnits);
}

// FP64 basis quantities, fixed-point shift and tables for one basis (whole workgroup; ends with a
// barrier).  Requires blockDim.x >= 256.
template <int COPIES, int COLS>
__device__ void p1_setup(P1Lds<COPIES, COLS>& S, const float* w, const P1Params& pp, bool zero_hist) {
    const int tid = threadIdx.x;
    if (zero_hist)
        for (int i = tid; i < 2 * kHistBins * COLS; i += blockDim.x) S.hist[i] = 0u;
    if (tid == 0) {
        derive_basis(w, pp.lambda, S.B);
        S.shift = table_shift(S.B, pp.i0, pp.hist_hi);
    }
    __syncthreads();
    const int u = S.shift;
    if (tid < kHistBins) {
        const int k = tid;
        const double sig0 = ldexp(256.0 / (double)pp.hist_hi[0], u), sig1 = ldexp(256.0 / (double)pp.hist_hi[1], u);
        for (int c = 0; c < 3; ++c) {
            const double od = S.B.ok ? od_u8((double)pp.i0[c], k) : 0.0;
            const int g = c == 0 ? kGuardUnits : 0;
            int4 e;
            e.x = __double2int_rn((S.B.pc[0][c] * od + (c == 0 ? S.B.pconst[0] : 0.0)) * sig0) + g;
            e.y = __double2int_rn((S.B.q[0][c] * od + (c == 0 ? S.B.fconst[0] : 0.0)) * sig0) + g;
            e.z = __double2int_rn((S.B.pc[1][c] * od + (c == 0 ? S.B.pconst[1] : 0.0)) * sig1) + g;
            e.w = __double2int_rn((S.B.q[1][c] * od + (c == 0 ? S.B.fconst[1] : 0.0)) * sig1) + g;
            for (int r = 0; r < COPIES; ++r) S.tab[(c * kHistBins + k) * COPIES + r] = e;
        }
    }
    __syncthreads();
}

// Counts the non-white pixels of units [0, cnt) of a chunk (buffer resource rs over the chunk's
// bytes) into the workgroup's LDS histogram.  `src_chunk` is the same chunk for the rare byte-wise
// re-reads.  Threads with tid >= nthreads do not participate (they must still call for barriers'
// sake only when the caller says so; this function has no barrier).
template <int COPIES, int COLS, int UNROLL>
__device__ void p1_chunk(P1Lds<COPIES, COLS>& S, const P1Params& pp, __amdgpu_buffer_rsrc_t rs,
                         const uint8_t* src_chunk, int cnt, int tid, int nthreads) {
    using L = P1Lds<COPIES, COLS>;
    const int lane = tid & 63;
    const int u = S.shift;
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const int32_t fmask = (1 << u) - 1;
    const uint32_t roff = (uint32_t)(lane & (COPIES - 1)) << 4;
    const char* tb = reinterpret_cast<const char*>(S.tab);
    uint32_t* h0 = S.hist + (lane & (COLS - 1));
    uint32_t* h1 = S.hist + kHistBins * COLS + (lane & (COLS - 1));
    const double sg0 = 256.0 / (double)pp.hist_hi[0], sg1 = 256.0 / (double)pp.hist_hi[1];

    auto entry = [&](int c, uint32_t k) -> int4 {
        return *reinterpret_cast<const int4*>(tb + c * L::kChannelBytes + ((k << L::kShift) | roff));
    };
    auto count_fixed = [&](int32_t x0, int32_t x1) {
        const int k0 = min(max(x0 >> u, 0), kHistBins - 1);
        const int k1 = min(max(x1 >> u, 0), kHistBins - 1);
        atomicAdd(h0 + k0 * COLS, 1u);
        atomicAdd(h1 + k1 * COLS, 1u);
    };
    // cold path: re-read one pixel, decide both bins in FP64 if it lies near a bin edge
    auto exact_pixel = [&](int64_t i, bool only_near) {
        const uint8_t* p = src_chunk + 3 * i;
        const uint32_t R = p[0], G = p[1], Bc = p[2];
        if ((int32_t)(R + G + Bc) >= thr) return;
        const int4 a = entry(0, R), b = entry(1, G), c = entry(2, Bc);
        const int32_t x0 = min(a.x + b.x + c.x, a.y + b.y + c.y);
        const int32_t x1 = min(a.z + b.z + c.z, a.w + b.w + c.w);
        const bool near = near_edge(x0, fmask) | near_edge(x1, fmask);
        if (near) {
            double d0, d1;
            solve64(S.B, od_u8((double)pp.i0[0], (int)R), od_u8((double)pp.i0[1], (int)G),
                    od_u8((double)pp.i0[2], (int)Bc), d0, d1);
            const double e0 = floor(d0 * sg0), e1 = floor(d1 * sg1);
            atomicAdd(h0 + (e0 >= 255.0 ? 255 : (int)e0) * COLS, 1u);
            atomicAdd(h1 + (e1 >= 255.0 ? 255 : (int)e1) * COLS, 1u);
        } else if (!only_near) {
            count_fixed(x0, x1);
        }
    };

    const int stride = nthreads * UNROLL;
    u32x3 cur[UNROLL];
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (int lb = tid; lb < cnt; lb += stride) {
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j)   // prefetch; past the chunk the loads return zeros
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb + stride + j * nthreads), 0, kLoadStream);
        bool any_near = false;
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            const bool valid = lb + j * nthreads < cnt;
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            bool tis[4];
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tis[q] = valid && (int32_t)(px[q][0] + px[q][1] + px[q][2]) < thr;
                any |= tis[q];
            }
            if (any) {
                // branch-free per pixel: every lane adds 0 or 1 (no exec-mask changes in the loop)
                int32_t x0[4], x1[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int4 a = entry(0, px[q][0]), b = entry(1, px[q][1]), c = entry(2, px[q][2]);
                    x0[q] = min(a.x + b.x + c.x, a.y + b.y + c.y);
                    x1[q] = min(a.z + b.z + c.z, a.w + b.w + c.w);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool near = near_edge(x0[q], fmask) | near_edge(x1[q], fmask);
                    any_near |= tis[q] & near;
                    const uint32_t inc = (tis[q] & !near) ? 1u : 0u;
                    const int k0 = min(max(x0[q] >> u, 0), kHistBins - 1);
                    const int k1 = min(max(x1[q] >> u, 0), kHistBins - 1);
                    atomicAdd(h0 + k0 * COLS, inc);
                    atomicAdd(h1 + k1 * COLS, inc);
                }
            }
        }
        if (any_near) {   // rare: settle this thread's near-edge pixels of the iteration in FP64
#pragma unroll 1
            for (int b = 0; b < 4 * UNROLL; ++b) {
                const int lu = lb + (b >> 2) * nthreads;
                if (lu < cnt) exact_pixel(4 * (int64_t)lu + (b & 3), true);
            }
        }
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) cur[j] = nxt[j];
    }
}

// Tail pixels (fewer than 4 after the last full unit) counted by one thread.
template <int COPIES, int COLS>
__device__ void p1_tail(P1Lds<COPIES, COLS>& S, const P1Params& pp, const uint8_t* px, int n) {
    using L = P1Lds<COPIES, COLS>;
    const int lane = threadIdx.x & 63;
    const int u = S.shift;
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const int32_t fmask = (1 << u) - 1;
    const uint32_t roff = (uint32_t)(lane & (COPIES - 1)) << 4;
    const char* tb = reinterpret_cast<const char*>(S.tab);
    uint32_t* h0 = S.hist + (lane & (COLS - 1));
    uint32_t* h1 = S.hist + kHistBins * COLS + (lane & (COLS - 1));
    for (int i = 0; i < n; ++i) {
        const uint32_t R = px[3 * i], G = px[3 * i + 1], Bc = px[3 * i + 2];
        if ((int32_t)(R + G + Bc) >= thr) continue;
        const int4 a = *reinterpret_cast<const int4*>(tb + ((R << L::kShift) | roff));
        const int4 b = *reinterpret_cast<const int4*>(tb + L::kChannelBytes + ((G << L::kShift) | roff));
        const int4 c = *reinterpret_cast<const int4*>(tb + 2 * L::kChannelBytes + ((Bc << L::kShift) | roff));
        const int32_t x0 = min(a.x + b.x + c.x, a.y + b.y + c.y);
        const int32_t x1 = min(a.z + b.z + c.z, a.w + b.w + c.w);
        int k0, k1;
        if (near_edge(x0, fmask) | near_edge(x1, fmask)) {
            double d0, d1;
            solve64(S.B, od_u8((double)pp.i0[0], (int)R), od_u8((double)pp.i0[1], (int)G),
                    od_u8((double)pp.i0[2], (int)Bc), d0, d1);
            const double e0 = floor(d0 * (256.0 / (double)pp.hist_hi[0])), e1 = floor(d1 * (256.0 / (double)pp.hist_hi[1]));
            k0 = e0 >= 255.0 ? 255 : (int)e0;
            k1 = e1 >= 255.0 ? 255 : (int)e1;
        } else {
            k0 = min(max(x0 >> u, 0), kHistBins - 1);
            k1 = min(max(x1 >> u, 0), kHistBins - 1);
        }
        atomicAdd(h0 + k0 * COLS, 1u);
        atomicAdd(h1 + k1 * COLS, 1u);
    }
}

// Adds the workgroup's LDS histogram to a global [2][256] uint64 histogram (ends with a barrier
// before, none after).
template <int COPIES, int COLS>
__device__ void p1_merge(P1Lds<COPIES, COLS>& S, unsigned long long* ghist) {
    __syncthreads();
    for (int t = threadIdx.x; t < 2 * kHistBins; t += blockDim.x) {
        const uint32_t* row = S.hist + t * COLS;
        uint32_t sum = 0;
        for (int l = 0; l < COLS; ++l) sum += row[(l + t) & (COLS - 1)];   // rotated: no bank conflicts
        if (sum) atomicAdd(ghist + t, (unsigned long long)sum);
    }
}

// ---------------------------------------------------------------- pass 1, byte-permute layout
// The same exact counting with a table layout chosen so that every LDS address is one v_perm_b32
// away from the pixel's dword: slot k (256 B) belongs to byte value k.  Two layouts:
//   wide (two 64 KB regions, 8 table copies, 16 histogram columns):
//     region 0: R entry copies in bank groups 0..7 (16 B each), G copies in groups 8..15
//     region 1: B copies in groups 4..11; histogram of bin k: stain 0 words col*4 (groups 0..3),
//               stain 1 words 192 + col*4 (groups 12..15)
//   A lane reads its pixel's three entries in a lane-dependent order and bank group (P1FLane's
//   schedule) such that the 16 lanes of every LDS cycle use 16 distinct bank groups: no bank
//   conflicts with 8 copies, where a fixed (R, G, B) order would meet pairwise in 8 groups.  The
//   sums are the same integer sums in another order.
//   narrow (one 64 KB region, 4 copies, 8 columns; two workgroups fit on a CU):
//     R copy r at r*16, G at 64 + r*16, B at 128 + r*16, histogram at 192 + j*32 + col*4  (r = lane & 3)
// An address is (value << 8) | (region << 16) | lane bits; the perm takes the value byte from the
// pixel's dword and the lane/region bytes from a per-lane constant.  With 2^16 fixed-point units
// (when the basis allows it, see table_shift) the bin is byte 2 of the clamped sum, so a bin
// address is one med3 + one perm.  Near-edge pixels are settled in FP64 (p1f_exact).
//
// The tables of this layout carry the guard shifted down by 2 * kGuardUnits: a sum y = x - 4 (x as
// in the other layout) is near an edge k >= 1 iff y >= 0 and its low u bits are >= 2^u - 4, i.e.
// iff (y & (sign | bits 2..u-1)) == bits 2..u-1, one AND and one compare.  Away from edges the bin
// of y equals the bin of x, so bins are taken from y directly.
template <bool WIDE>
struct P1FLayout {
    static constexpr int kCopies = WIDE ? 8 : 4;
    static constexpr int kCols = WIDE ? 16 : 8;
    static constexpr uint32_t kBytes = WIDE ? 2u * kHistBins * 256u : kHistBins * 256u;
    static constexpr uint32_t kG = WIDE ? 128u : 64u;              // G entries within the slot
    static constexpr uint32_t kBRegion = WIDE ? 0x10000u : 0u;     // region of the B entries
    static constexpr uint32_t kB = WIDE ? 64u : 128u;              // B entries within the slot
    static constexpr uint32_t kHRegion = WIDE ? 0x10000u : 0u;     // region of the histogram
    static constexpr uint32_t kH = WIDE ? 0u : 192u;               // histogram words within the slot
    static constexpr uint32_t kStain1 = WIDE ? 192u : 4u * kCols;  // stain 1's columns after stain 0's
    // word index of histogram word i (0 .. 2 kCols - 1: stain i / kCols, column i % kCols) of bin k
    static __device__ __forceinline__ uint32_t hist_word(uint32_t k, uint32_t i) {
        return (kHRegion + k * 256u + kH + (i / kCols) * kStain1) / 4u + i % kCols;
    }
};

template <bool WIDE>
struct P1FLds {
    int4 mem[P1FLayout<WIDE>::kBytes / 16];
    double od[3][kHistBins];        // FP64 optical densities of Eq. 1 for the near-edge path
    Basis64 B;
    int shift;                      // fixed-point resolution u (<= 16)
};

// selector placing byte p of S0 in byte 1, S1's bytes 0 and 2 in bytes 0 and 2, zero in byte 3
__device__ __forceinline__ constexpr uint32_t perm_sel(int p) { return 0x0c020000u | ((uint32_t)(4 + p) << 8); }

__device__ __forceinline__ uint32_t p1f_hist_addr(int bin, uint32_t lh) { return ((uint32_t)bin << 8) | lh; }

template <bool WIDE>
__device__ void p1f_setup(P1FLds<WIDE>& S, const float* w, const P1Params& pp, bool zero_hist) {
    using Y = P1FLayout<WIDE>;
    const int tid = threadIdx.x;
    uint32_t* words = reinterpret_cast<uint32_t*>(S.mem);
    if (zero_hist) {
        constexpr int per = 2 * Y::kCols;     // histogram words per slot
        for (int i = tid; i < kHistBins * per; i += blockDim.x) words[Y::hist_word(i / per, i % per)] = 0u;
    }
    if (tid == 0) {
        derive_basis(w, pp.lambda, S.B);
        const int u = table_shift(S.B, pp.i0, pp.hist_hi);
        S.shift = u < 16 ? u : 16;
    }
    __syncthreads();
    const int u = S.shift;
    if (tid < kHistBins) {
        const int k = tid;
        const double sig0 = ldexp(256.0 / (double)pp.hist_hi[0], u), sig1 = ldexp(256.0 / (double)pp.hist_hi[1], u);
        char* base = reinterpret_cast<char*>(S.mem);
        for (int c = 0; c < 3; ++c) S.od[c][k] = od_u8((double)pp.i0[c], k);
        for (int c = 0; c < 3; ++c) {
            const double od = S.B.ok ? S.od[c][k] : 0.0;
            const int g = c == 0 ? kGuardUnits - 2 * kGuardUnits : 0;   // shifted guard (see above)
            int4 e;
            e.x = __double2int_rn((S.B.pc[0][c] * od + (c == 0 ? S.B.pconst[0] : 0.0)) * sig0) + g;
            e.y = __double2int_rn((S.B.q[0][c] * od + (c == 0 ? S.B.fconst[0] : 0.0)) * sig0) + g;
            e.z = __double2int_rn((S.B.pc[1][c] * od + (c == 0 ? S.B.pconst[1] : 0.0)) * sig1) + g;
            e.w = __double2int_rn((S.B.q[1][c] * od + (c == 0 ? S.B.fconst[1] : 0.0)) * sig1) + g;
            const uint32_t off = (c == 0 ? 0u : c == 1 ? Y::kG : (Y::kBRegion | Y::kB)) + ((uint32_t)k << 8);
            for (int r = 0; r < Y::kCopies; ++r) *reinterpret_cast<int4*>(base + off + r * 16) = e;
        }
    }
    __syncthreads();
}

// Near-edge test of a shifted sum y (see the layout comment); nmask = sign | bits 2..u-1.
__device__ __forceinline__ uint32_t p1f_nmask(int u) { return 0x80000000u | ((((1u << u) - 1u)) & ~3u); }
__device__ __forceinline__ bool p1f_near(int32_t y, uint32_t nmask) {
    return ((uint32_t)y & nmask) == (nmask & 0x7FFFFFFFu);
}

// FP64 decision for one pixel known to be non-white; adds to the exact bins.
template <bool WIDE>
__device__ __forceinline__ void p1f_exact(P1FLds<WIDE>& S, const P1Params& pp, uint32_t R, uint32_t G, uint32_t Bc,
                                          uint32_t lh) {
    double d0, d1;
    solve64(S.B, S.od[0][R], S.od[1][G], S.od[2][Bc], d0, d1);
    const double e0 = floor(d0 * (256.0 / (double)pp.hist_hi[0])), e1 = floor(d1 * (256.0 / (double)pp.hist_hi[1]));
    char* base = reinterpret_cast<char*>(S.mem);
    atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_hist_addr(e0 >= 255.0 ? 255 : (int)e0, lh)), 1u);
    atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_hist_addr(e1 >= 255.0 ? 255 : (int)e1, lh) +
                                          P1FLayout<WIDE>::kStain1), 1u);
}

// Fixed-point (shifted) sums of one pixel from its three bytes (cold path and tail).
template <bool WIDE>
__device__ __forceinline__ void p1f_sums(const P1FLds<WIDE>& S, uint32_t R, uint32_t G, uint32_t Bc, uint32_t r16,
                                         int32_t& x0, int32_t& x1) {
    using Y = P1FLayout<WIDE>;
    const char* base = reinterpret_cast<const char*>(S.mem);
    const int4 a = *reinterpret_cast<const int4*>(base + ((R << 8) | r16));
    const int4 b = *reinterpret_cast<const int4*>(base + ((G << 8) | r16) + Y::kG);
    const int4 c = *reinterpret_cast<const int4*>(base + (Y::kBRegion | (Bc << 8) | r16) + Y::kB);
    x0 = min(a.x + b.x + c.x, a.y + b.y + c.y);
    x1 = min(a.z + b.z + c.z, a.w + b.w + c.w);
}

// Per-lane constants of the byte-permute layout.  Wide layout: read k (0..2) of a pixel takes
// channel ch (0 R, 1 G, 2 B) from bank group g, by quad q = (lane & 15) >> 2 and j = lane & 3:
//   q = 0: B in 4+j, R in j,    G in 8+j        q = 2: R in j,    B in 4+j, G in 12+j
//   q = 1: B in 8+j, G in 12+j, R in 4+j        q = 3: G in 12+j, B in 8+j, R in j
// In each read the 16 lanes of a cycle use groups 0..15 once (R copies live in groups 0..7 and G in
// 8..15 of region 0, B in 4..11 of region 1).  lk[k] holds the read's region and group, sel[k] the
// perm selector of its channel's byte in a dword holding the pixel as (R, G, B) in bytes 0..2, selz[k]
// in one holding it in bytes 1..3.
// wa is 2^32 - thr (thr the white-sum threshold, 2^31 - 1 without one) for p1f_bins, kept in a vector
// register for the whole run: the byte dot product that takes it has its weights in a scalar register
// and can read only one scalar operand.
struct P1FLane {
    uint32_t lane, r16, la, lb, lh, lh1, wa;
    uint32_t lk[3], sel[3], selz[3];
};

template <bool WIDE>
__device__ __forceinline__ P1FLane p1f_lane(int tid, int32_t white_sum) {
    using Y = P1FLayout<WIDE>;
    P1FLane L;
    L.lane = (uint32_t)(tid & 63);
    L.wa = 0u - (uint32_t)(white_sum > 0 ? white_sum : 0x7FFFFFFF);
    __asm__("" : "+v"(L.wa));
    L.r16 = (uint32_t)(tid & (Y::kCopies - 1)) << 4;
    L.la = L.r16;
    L.lb = Y::kBRegion | L.r16;
    L.lh = Y::kHRegion | (Y::kH + ((uint32_t)(tid & (Y::kCols - 1)) << 2));   // stain 0 column word
    L.lh1 = L.lh + Y::kStain1;                                                 // stain 1
    const int q = (tid & 15) >> 2, j = tid & 3;
    const int ch = (q == 0 ? 0x102 : q == 1 ? 0x012 : q == 2 ? 0x120 : 0x021);   // channel of read k: nibble k
    const int gb = (q == 0 ? 0x804 : q == 1 ? 0x4C8 : q == 2 ? 0xC40 : 0x08C);   // group base of read k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int c = (ch >> (4 * k)) & 15, g = ((gb >> (4 * k)) & 15) + j;
        L.lk[k] = (c == 2 ? Y::kBRegion : 0u) | ((uint32_t)g << 4);
        L.sel[k] = perm_sel(c);
        L.selz[k] = perm_sel(c + 1);
    }
    return L;
}

// Fixed-point sums (shifted guard, see above) of the four pixels of a unit (dwords X, Y0, Z).
template <bool WIDE>
__device__ __forceinline__ void p1f_unit_sums(const P1FLds<WIDE>& S, const P1FLane& L, uint32_t X, uint32_t Y0,
                                              uint32_t Z, int32_t (&y0)[4], int32_t (&y1)[4]) {
    using Y = P1FLayout<WIDE>;
    const char* base = reinterpret_cast<const char*>(S.mem);
    auto rd = [&](uint32_t addr) -> int4 { return *reinterpret_cast<const int4*>(base + addr); };
    if constexpr (WIDE) {
        // pixels 1 and 2 gathered as (R, G, B, 0); pixel 0 is bytes 0..2 of X, pixel 3 bytes 1..3 of Z
        const uint32_t w[3] = {X, __builtin_amdgcn_perm(Y0, X, 0x0c050403u), __builtin_amdgcn_perm(Z, Y0, 0x0c040302u)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 e[3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                e[k] = rd(q < 3 ? __builtin_amdgcn_perm(w[q], L.lk[k], L.sel[k]) : __builtin_amdgcn_perm(Z, L.lk[k], L.selz[k]));
            y0[q] = min(e[0].x + e[1].x + e[2].x, e[0].y + e[1].y + e[2].y);
            y1[q] = min(e[0].z + e[1].z + e[2].z, e[0].w + e[1].w + e[2].w);
        }
    } else {
        const uint32_t aR[4] = {__builtin_amdgcn_perm(X, L.la, perm_sel(0)), __builtin_amdgcn_perm(X, L.la, perm_sel(3)),
                                __builtin_amdgcn_perm(Y0, L.la, perm_sel(2)), __builtin_amdgcn_perm(Z, L.la, perm_sel(1))};
        const uint32_t aG[4] = {__builtin_amdgcn_perm(X, L.la, perm_sel(1)), __builtin_amdgcn_perm(Y0, L.la, perm_sel(0)),
                                __builtin_amdgcn_perm(Y0, L.la, perm_sel(3)), __builtin_amdgcn_perm(Z, L.la, perm_sel(2))};
        const uint32_t aB[4] = {__builtin_amdgcn_perm(X, L.lb, perm_sel(2)), __builtin_amdgcn_perm(Y0, L.lb, perm_sel(1)),
                                __builtin_amdgcn_perm(Z, L.lb, perm_sel(0)), __builtin_amdgcn_perm(Z, L.lb, perm_sel(3))};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 a = rd(aR[q]), b = rd(aG[q] + Y::kG), c = rd(aB[q] + Y::kB);
            y0[q] = min(a.x + b.x + c.x, a.y + b.y + c.y);
            y1[q] = min(a.z + b.z + c.z, a.w + b.w + c.w);
        }
    }
}

// R + G + B of the four pixels of a unit (byte dot products; pixels 1 and 2 from the same gathered
// dwords as the wide layout's table addresses, which the compiler shares).
__device__ __forceinline__ void p1f_white_sums(uint32_t X, uint32_t Y0, uint32_t Z, int32_t (&sum)[4]) {
    sum[0] = (int32_t)__builtin_amdgcn_udot4(X, 0x00010101u, 0u, false);
    sum[1] = (int32_t)__builtin_amdgcn_udot4(__builtin_amdgcn_perm(Y0, X, 0x0c050403u), 0x00010101u, 0u, false);
    sum[2] = (int32_t)__builtin_amdgcn_udot4(__builtin_amdgcn_perm(Z, Y0, 0x0c040302u), 0x00010101u, 0u, false);
    sum[3] = (int32_t)__builtin_amdgcn_udot4(Z, 0x01010100u, 0u, false);
}

// Histogram bin address of a fixed-point candidate sum (shifted guard, see the layout comment).
template <bool WIDE, bool U16>
__device__ __forceinline__ uint32_t p1f_bin_addr(const P1FLds<WIDE>& S, int32_t y, uint32_t lh) {
    return U16 ? __builtin_amdgcn_perm((uint32_t)min(max(y, 0), 0xFFFFFF), lh, perm_sel(2))
               : p1f_hist_addr(min(max(y >> S.shift, 0), kHistBins - 1), lh);
}

// Histogram adds of one unit per active lane from its pixel dwords and fixed-point candidate sums.
// One edge test per unit: a unit with any of its 8 candidate sums near a bin edge is left out here
// (its lane skips the adds) and settled whole by p1f_settle (rare); returns those lanes.  A pixel's
// increment is bit 31 of R + G + B + L.wa = R + G + B + 2^32 - thr (one byte dot product; with
// 0 < thr < 2^31 and R + G + B <= 765 the sum wraps below 2^31 exactly when R + G + B >= thr, a white
// pixel).
template <bool WIDE, bool U16>
__device__ __forceinline__ uint64_t p1f_bins(P1FLds<WIDE>& S, const P1FLane& L, uint32_t X, uint32_t Y0, uint32_t Z,
                                             const int32_t (&y0)[4], const int32_t (&y1)[4], uint32_t nmask,
                                             uint64_t valid_lanes) {
    char* base = reinterpret_cast<char*>(S.mem);
    // k(y) is 0 exactly when y is near an edge (p1f_near), so the unit is near one iff the minimum is 0
    const uint32_t nv = nmask & 0x7FFFFFFFu;
    auto k = [&](int32_t y) { return ((uint32_t)y & nmask) ^ nv; };
    const uint32_t m0 = min(min(k(y0[0]), k(y0[1])), min(k(y0[2]), k(y0[3])));
    const uint32_t m1 = min(min(k(y1[0]), k(y1[1])), min(k(y1[2]), k(y1[3])));
    const uint64_t nearm = __ballot(min(m0, m1) == 0u) & valid_lanes;
    if (!__builtin_amdgcn_inverse_ballot_w64(nearm)) {
        // the pixels as (R, G, B, 0) dwords (1 and 2 gathered as for the table addresses); pixel 3 is
        // bytes 1..3 of Z
        const uint32_t px[4] = {X, __builtin_amdgcn_perm(Y0, X, 0x0c050403u), __builtin_amdgcn_perm(Z, Y0, 0x0c040302u),
                                Z};
        const uint32_t wt[4] = {0x00010101u, 0x00010101u, 0x00010101u, 0x01010100u};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t inc = __builtin_amdgcn_udot4(px[q], wt[q], L.wa, false) >> 31;
            atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_bin_addr<WIDE, U16>(S, y0[q], L.lh)), inc);
            atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_bin_addr<WIDE, U16>(S, y1[q], L.lh1)), inc);
        }
    }
    return nearm;
}

// Counts the non-white pixels of the units p1f_bins left out (lanes in nearm; rare): a pixel near a
// bin edge in FP64, the others by their fixed-point bins.
template <bool WIDE, bool U16>
__device__ __forceinline__ void p1f_settle(P1FLds<WIDE>& S, const P1Params& pp, const P1FLane& L, uint32_t X,
                                           uint32_t Y0, uint32_t Z, uint64_t nearm, int32_t thr, uint32_t nmask) {
    if (nearm && __builtin_amdgcn_inverse_ballot_w64(nearm)) {
        char* base = reinterpret_cast<char*>(S.mem);
        u32x3 un;
        un.x = X; un.y = Y0; un.z = Z;
        uint32_t px[4][3];
        bytes_of_unit(un, px);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t R = px[q][0], G = px[q][1], Bc = px[q][2];
            if ((int32_t)(R + G + Bc) >= thr) continue;
            int32_t y0, y1;
            p1f_sums(S, R, G, Bc, L.r16, y0, y1);
            if (p1f_near(y0, nmask) | p1f_near(y1, nmask)) {
                p1f_exact(S, pp, R, G, Bc, L.lh);
            } else {
                atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_bin_addr<WIDE, U16>(S, y0, L.lh)), 1u);
                atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_bin_addr<WIDE, U16>(S, y1, L.lh1)), 1u);
            }
        }
    }
}

// Counts the non-white pixels of one unit per lane (dwords X, Y0, Z) on the lanes where `valid`, and
// settles the unit's near-edge pixels in FP64 right away (rare; only on the lanes that hold one).
template <bool WIDE, bool U16>
__device__ __forceinline__ void p1f_count(P1FLds<WIDE>& S, const P1Params& pp, const P1FLane& L, uint32_t X,
                                          uint32_t Y0, uint32_t Z, bool valid) {
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const uint32_t nmask = p1f_nmask(U16 ? 16 : S.shift);
    const uint64_t valid_lanes = __ballot(valid);
    uint64_t nearm = 0;       // lanes with a near-edge non-white pixel
    if (valid) {
        int32_t y0[4], y1[4];
        p1f_unit_sums(S, L, X, Y0, Z, y0, y1);
        nearm = p1f_bins<WIDE, U16>(S, L, X, Y0, Z, y0, y1, nmask, valid_lanes);
    }
    p1f_settle<WIDE, U16>(S, pp, L, X, Y0, Z, nearm, thr, nmask);
}

// Units with a non-white pixel waiting for a full wavefront of counting work (wide layout): lanes
// 0 .. n-1 of u hold one each; n is the same in every lane.
struct P1FPend {
    u32x3 u;
    int n;
};

__device__ __forceinline__ P1FPend p1f_pend() {
    P1FPend P;
    P.u.x = 0u; P.u.y = 0u; P.u.z = 0u;
    P.n = 0;
    return P;
}

// Counts the non-white pixels among UNROLL units of one thread: unit j is unit lb0 + j * nthreads
// of a run of cnt units (cur holds their bytes).  Every lane of the wavefront must be active.
//
// A wavefront pays for an LDS or vector instruction whatever its exec mask, and inside tissue most
// 256-pixel spans mix units with and without tissue, so with the wide layout the units that hold a
// non-white pixel are packed into full wavefronts first: the units of one slot j are permuted
// (ds_permute_b32, a full permutation of the 64 lanes: tissue units to lanes n, n+1, ... modulo 64
// in lane order, the others to the remaining lanes) and merged into the pending units P; whenever 64
// are pending they are counted as one wavefront.  The caller counts what is left with p1f_flush.
template <bool WIDE, int UNROLL, bool U16>
__device__ __forceinline__ void p1f_units(P1FLds<WIDE>& S, const P1Params& pp, const P1FLane& L,
                                          const u32x3 (&cur)[UNROLL], int lb0, int cnt, int nthreads, P1FPend& P) {
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) {
        const bool valid = lb0 + j * nthreads < cnt;
        const uint32_t X = cur[j].x, Y0 = cur[j].y, Z = cur[j].z;
        const int32_t s0 = (int32_t)__builtin_amdgcn_udot4(X, 0x00010101u, 0u, false);
        const int32_t s1 = (int32_t)__builtin_amdgcn_udot4(Y0, 0x00000101u, __builtin_amdgcn_udot4(X, 0x01000000u, 0u, false), false);
        const int32_t s2 = (int32_t)__builtin_amdgcn_udot4(Z, 0x00000001u, __builtin_amdgcn_udot4(Y0, 0x01010000u, 0u, false), false);
        const int32_t s3 = (int32_t)__builtin_amdgcn_udot4(Z, 0x01010100u, 0u, false);
        const bool tissue = valid && min(min(s0, s1), min(s2, s3)) < thr;   // a non-white pixel in the unit
        if constexpr (!WIDE) {
            p1f_count<WIDE, U16>(S, pp, L, X, Y0, Z, tissue);
        } else {
            const uint64_t m = __ballot(tissue);
            if (m == 0) continue;
            const int c = __popcll(m);
            P.n = __builtin_amdgcn_readfirstlane(P.n);   // uniform by construction: keep it scalar
            if (c == 64 && P.n == 0) {   // a full wavefront as it is
                p1f_count<WIDE, U16>(S, pp, L, X, Y0, Z, true);
                continue;
            }
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            const uint32_t n0 = (uint32_t)P.n;
            const uint32_t to_t = n0 + r, to_w = n0 + (uint32_t)c + L.lane - r;
            // byte address; ds_permute_b32 takes the destination lane modulo 64
            const uint32_t dst = (__builtin_amdgcn_inverse_ballot_w64(m) ? to_t : to_w) << 2;
            u32x3 v;
            v.x = (uint32_t)__builtin_amdgcn_ds_permute((int)dst, (int)X);
            v.y = (uint32_t)__builtin_amdgcn_ds_permute((int)dst, (int)Y0);
            v.z = (uint32_t)__builtin_amdgcn_ds_permute((int)dst, (int)Z);
            const int e = __builtin_amdgcn_readfirstlane(P.n + c);
            if (e < 64) {
                const bool take = L.lane >= n0 && L.lane < (uint32_t)e;
                P.u.x = take ? v.x : P.u.x;
                P.u.y = take ? v.y : P.u.y;
                P.u.z = take ? v.z : P.u.z;
                P.n = e;
            } else {
                const bool take = L.lane >= n0;
                P.u.x = take ? v.x : P.u.x;
                P.u.y = take ? v.y : P.u.y;
                P.u.z = take ? v.z : P.u.z;
                p1f_count<WIDE, U16>(S, pp, L, P.u.x, P.u.y, P.u.z, true);
                P.u = v;                 // lanes 0 .. e - 65 hold the units that did not fit
                P.n = e - 64;
            }
        }
    }
}

// Counts the pending units (a partial wavefront) and empties P.
template <bool WIDE, bool U16>
__device__ __forceinline__ void p1f_flush(P1FLds<WIDE>& S, const P1Params& pp, const P1FLane& L, P1FPend& P) {
    P.n = __builtin_amdgcn_readfirstlane(P.n);
    if (WIDE && P.n > 0) p1f_count<WIDE, U16>(S, pp, L, P.u.x, P.u.y, P.u.z, L.lane < (uint32_t)P.n);
    P.n = 0;
}

// Contiguous run of cnt units (buffer resource rs over its bytes): each thread takes units tid,
// tid + nthreads, ..., UNROLL of them per iteration with one iteration of prefetch.  Nothing for
// cnt <= 0.
template <bool WIDE, int UNROLL, bool U16>
__device__ void p1f_run(P1FLds<WIDE>& S, const P1Params& pp, __amdgpu_buffer_rsrc_t rs, int cnt, int tid,
                        int nthreads) {
    if (cnt <= 0) return;
    const P1FLane L = p1f_lane<WIDE>(tid, pp.white_sum);
    const int stride = nthreads * UNROLL;
    P1FPend P = p1f_pend();
    int b0 = 0;                                // the same trip count in every lane
    // one iteration: the next iteration's loads into nxt (past the run they return zeros), then cur
    auto step = [&](const u32x3 (&cur)[UNROLL], u32x3 (&nxt)[UNROLL]) {
        const int lb0 = b0 + tid;
#pragma unroll
        for (int j = 0; j < UNROLL; ++j)
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb0 + stride + j * nthreads), 0, kLoadStream);
        p1f_units<WIDE, UNROLL, U16>(S, pp, L, cur, lb0, cnt, nthreads, P);
        b0 += stride;
    };
    u32x3 ua[UNROLL], ub[UNROLL];              // two buffers taking turns, so no register copies
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) ua[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (;;) {
        step(ua, ub);
        if (b0 >= cnt) break;
        step(ub, ua);
        if (b0 >= cnt) break;
    }
    p1f_flush<WIDE, U16>(S, pp, L, P);
}

// Grid-stride form: the image's units form tiles of nthreads * UNROLL units.  Workgroup b takes the
// tiles of sequence positions b, b + gridDim.x, ...; position t holds tile (t * scatter) mod n_tiles.
// With scatter = 1 the grid sweeps the image front to back; a scatter near 0.618 n_tiles (coprime
// with n_tiles, so the map is a permutation) spreads the tiles in flight over the whole image, so
// compute-heavy tissue tiles and memory-bound background tiles run side by side instead of in
// alternating phases.  step = (gridDim.x * scatter) mod n_tiles advances a workgroup's tile.
template <bool WIDE, int UNROLL, bool U16>
__device__ void p1f_tiles(P1FLds<WIDE>& S, const P1Params& pp, const uint8_t* src, int64_t n_units, int tid,
                          int nthreads, int64_t scatter, int64_t step) {
    const P1FLane L = p1f_lane<WIDE>(tid, pp.white_sum);
    const int64_t tu = (int64_t)nthreads * UNROLL;
    const int64_t n_tiles = (n_units + tu - 1) / tu;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    int64_t ph = (t * scatter) % n_tiles;       // tile at sequence position t
    auto tile_rs = [&](int64_t tt, int64_t tile) {   // one descriptor built from selected fields (stays scalar)
        const bool in = tt < n_tiles;
        return chunk_rsrc(src, in ? tile * tu : 0, in ? min(tu, n_units - tile * tu) : 0);
    };
    P1FPend P = p1f_pend();
    // one tile: the next tile's loads into nxt, then the units of cur
    auto tile_step = [&](const u32x3 (&cur)[UNROLL], u32x3 (&nxt)[UNROLL]) {
        int64_t pn = ph + step;
        if (pn >= n_tiles) pn -= n_tiles;
        const __amdgpu_buffer_rsrc_t rn = tile_rs(t + gridDim.x, pn);   // empty past the end: loads return zeros
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * nthreads), 0, kLoadStream);
        const int cnt = (int)min(tu, n_units - ph * tu);
        p1f_units<WIDE, UNROLL, U16>(S, pp, L, cur, tid, cnt, nthreads, P);
        ph = pn;
        t += gridDim.x;
    };
    u32x3 ua[UNROLL], ub[UNROLL];   // two buffers taking turns, so no register copies between tiles
    const __amdgpu_buffer_rsrc_t rs = tile_rs(t, ph);
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) ua[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (;;) {
        tile_step(ua, ub);
        if (t >= n_tiles) break;
        tile_step(ub, ua);
        if (t >= n_tiles) break;
    }
    p1f_flush<WIDE, U16>(S, pp, L, P);
}

// Multiplier of the tile permutation above: 1 when the grid covers every tile at once, else the
// first integer from floor(0.618 n_tiles) up that is coprime with n_tiles.
inline int64_t tile_scatter(int64_t n_tiles, int64_t grid) {
    if (n_tiles <= grid || n_tiles < 3) return 1;
    auto gcd = [](int64_t a, int64_t b) { while (b) { const int64_t r = a % b; a = b; b = r; } return a; };
    int64_t k = (int64_t)(0.6180339887498949 * (double)n_tiles);
    while (gcd(k, n_tiles) != 1) ++k;
    return k;
}

// Tail pixels (fewer than 4 after the last full unit) counted by one thread.
template <bool WIDE>
__device__ void p1f_tail(P1FLds<WIDE>& S, const P1Params& pp, const uint8_t* px, int n) {
    const int u = S.shift;
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const uint32_t nmask = p1f_nmask(u);
    const P1FLane L = p1f_lane<WIDE>(threadIdx.x, pp.white_sum);
    char* base = reinterpret_cast<char*>(S.mem);
    for (int i = 0; i < n; ++i) {
        const uint32_t R = px[3 * i], G = px[3 * i + 1], Bc = px[3 * i + 2];
        if ((int32_t)(R + G + Bc) >= thr) continue;
        int32_t y0, y1;
        p1f_sums(S, R, G, Bc, L.r16, y0, y1);
        if (p1f_near(y0, nmask) | p1f_near(y1, nmask)) {
            p1f_exact(S, pp, R, G, Bc, L.lh);
        } else {
            atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_hist_addr(min(max(y0 >> u, 0), kHistBins - 1), L.lh)), 1u);
            atomicAdd(reinterpret_cast<uint32_t*>(base + p1f_hist_addr(min(max(y1 >> u, 0), kHistBins - 1), L.lh1)), 1u);
        }
    }
}

// Adds the workgroup's LDS histogram to a global [2][256] uint64 histogram (barrier before).
template <bool WIDE>
__device__ void p1f_merge(P1FLds<WIDE>& S, unsigned long long* ghist) {
    using Y = P1FLayout<WIDE>;
    __syncthreads();
    const uint32_t* words = reinterpret_cast<const uint32_t*>(S.mem);
    for (int t = threadIdx.x; t < 2 * kHistBins; t += blockDim.x) {
        const int j = t >> 8, k = t & (kHistBins - 1);
        const uint32_t* row = words + (Y::kHRegion + (uint32_t)k * 256u + Y::kH + (uint32_t)j * Y::kStain1) / 4;
        uint32_t sum = 0;
        for (int l = 0; l < Y::kCols; ++l) sum += row[(l + t) & (Y::kCols - 1)];   // rotated: no bank conflicts
        if (sum) atomicAdd(ghist + t, (unsigned long long)sum);
    }
}

// ================================================================================== percentile

struct FinalShared {
    uint64_t cum[2][kHistBins];
    double P[2];
    int kstar[2];
};

// Eq. (3) percentile of both stains from a [2][256] histogram (any blockDim >= 256).  Afterwards
// F.P[j] and F.kstar[j] (-1: no tissue) are valid on every thread.
__device__ inline void block_percentiles(const uint64_t* hist, double q, const float hist_hi[2], FinalShared& F) {
    const int t = threadIdx.x;
    if (t < kHistBins) {
        F.cum[0][t] = hist[t];
        F.cum[1][t] = hist[kHistBins + t];
    }
    if (t < 2) { F.P[t] = 0.0; F.kstar[t] = -1; }
    __syncthreads();
    for (int off = 1; off < kHistBins; off <<= 1) {
        uint64_t v0 = 0, v1 = 0;
        if (t < kHistBins && t >= off) { v0 = F.cum[0][t - off]; v1 = F.cum[1][t - off]; }
        __syncthreads();
        if (t < kHistBins) { F.cum[0][t] += v0; F.cum[1][t] += v1; }
        __syncthreads();
    }
    if (t < kHistBins) {
        for (int j = 0; j < 2; ++j) {
            double P;
            if (percentile_owner(F.cum[j], t, q, (double)hist_hi[j], P)) { F.P[j] = P; F.kstar[j] = t; }
        }
    }
    __syncthreads();
}

__device__ inline int stain_flags(const FinalShared& F, int j, bool basis_ok) {
    int fl = 0;
    if (F.kstar[j] < 0) fl |= SPCN_FLAG_NO_TISSUE;
    if (F.kstar[j] == kHistBins - 1) fl |= SPCN_FLAG_RANGE;
    if (F.kstar[j] == 0) fl |= SPCN_FLAG_BIN0;
    if (!basis_ok) fl |= SPCN_FLAG_BASIS;
    return fl;
}

// A target scale that is not finite and positive (NaN fails both compares) is refused.
__device__ inline int scale_flag(float scale_tgt) {
    return (scale_tgt > 0.0f && scale_tgt < __builtin_huge_valf()) ? 0 : SPCN_FLAG_SCALE;
}

// Scale of Eq. (3): no tissue, a percentile in bin 0 or a refused target scale keeps the density
// unscaled.
__device__ inline double stain_scale(double scale_tgt, double P, int fl) {
    if ((fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0 | SPCN_FLAG_SCALE)) || !(P > 0.0)) return 1.0;
    return scale_tgt / P;
}

// ================================================================================== pass 2

// Per-launch (or per-tile) recolouring constants: y_c = exp2(L_c - M_c0 h0 - M_c1 h1).
struct RecolourConsts {
    float M[3][2];      // log2(e) * W_tgt[c, j] * s_j
    float L[3];         // log2(i0_out[c])
    float a0, a1;       // g01 / g00, g01 / g11 of the source basis
};

__device__ inline void make_recolour(RecolourConsts& K, const float* w_tgt, const double s[2], const float i0_out[3],
                                     const Basis64& B) {
    for (int c = 0; c < 3; ++c) {
        for (int j = 0; j < 2; ++j) K.M[c][j] = (float)(kLog2e * (double)w_tgt[c + 3 * j] * s[j]);
        K.L[c] = (float)log2((double)i0_out[c]);
    }
    K.a0 = (float)B.a[0];
    K.a1 = (float)B.a[1];
}

// The constants moved to scalar registers (they are the same in every lane), which keeps ~11 vector
// registers free in the recolour loops.
__device__ __forceinline__ RecolourConsts uniform_consts(const RecolourConsts& K) {
    RecolourConsts R;
    auto u = [](float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); };
    for (int c = 0; c < 3; ++c) {
        R.M[c][0] = u(K.M[c][0]);
        R.M[c][1] = u(K.M[c][1]);
        R.L[c] = u(K.L[c]);
    }
    R.a0 = u(K.a0);
    R.a1 = u(K.a1);
    return R;
}

template <int COPIES>
struct P2Lds {
    static_assert((COPIES & (COPIES - 1)) == 0, "power of two");
    static constexpr int kChannelBytes = kHistBins * COPIES * 8;
    static constexpr int kShift = ilog2(COPIES * 8);
    float2 ftab[3 * kHistBins * COPIES];   // (f0, f1) in density units, entry k copy r at k*COPIES + r
};

// FP32 density tables of pass 2 for one basis (threads 0..255 each build one intensity; barrier).
template <int COPIES>
__device__ void p2_tables(P2Lds<COPIES>& T, const Basis64& B, const float i0[3]) {
    const int k = threadIdx.x;
    if (k < kHistBins) {
        for (int c = 0; c < 3; ++c) {
            const double od = B.ok ? od_u8((double)i0[c], k) : 0.0;
            float2 f;
            f.x = (float)(B.q[0][c] * od + (c == 0 ? B.fconst[0] : 0.0));
            f.y = (float)(B.q[1][c] * od + (c == 0 ? B.fconst[1] : 0.0));
            for (int r = 0; r < COPIES; ++r) T.ftab[(c * kHistBins + k) * COPIES + r] = f;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t recolour_byte(float h0, float h1, const RecolourConsts& K, int c, uint32_t sel,
                                                  uint32_t acc) {
    float z = fmaf(-K.M[c][0], h0, K.L[c]);
    z = fmaf(-K.M[c][1], h1, z);
    return __builtin_amdgcn_cvt_pk_u8_f32(__builtin_amdgcn_exp2f(z), sel, acc);
}

// Densities of one pixel from the FP32 tables (h_j = max(0, f_j + a_j min(f_other, 0))).
template <int COPIES>
__device__ __forceinline__ void p2_densities(const P2Lds<COPIES>& T, uint32_t roff, const RecolourConsts& K,
                                             uint32_t R, uint32_t G, uint32_t Bc, float& h0, float& h1) {
    using L = P2Lds<COPIES>;
    const char* tb = reinterpret_cast<const char*>(T.ftab);
    const float2 r = *reinterpret_cast<const float2*>(tb + ((R << L::kShift) | roff));
    const float2 g = *reinterpret_cast<const float2*>(tb + L::kChannelBytes + ((G << L::kShift) | roff));
    const float2 b = *reinterpret_cast<const float2*>(tb + 2 * L::kChannelBytes + ((Bc << L::kShift) | roff));
    const float f0 = r.x + g.x + b.x, f1 = r.y + g.y + b.y;
    h0 = fmaxf(0.0f, fmaf(K.a0, fminf(f1, 0.0f), f0));   // tables are zero for a singular basis
    h1 = fmaxf(0.0f, fmaf(K.a1, fminf(f0, 0.0f), f1));
}

__device__ __forceinline__ u32x3 recolour_unit(const float h0[4], const float h1[4], const RecolourConsts& K) {
    uint32_t o0 = 0, o1 = 0, o2 = 0;
    o0 = recolour_byte(h0[0], h1[0], K, 0, 0, o0);
    o0 = recolour_byte(h0[0], h1[0], K, 1, 1, o0);
    o0 = recolour_byte(h0[0], h1[0], K, 2, 2, o0);
    o0 = recolour_byte(h0[1], h1[1], K, 0, 3, o0);
    o1 = recolour_byte(h0[1], h1[1], K, 1, 0, o1);
    o1 = recolour_byte(h0[1], h1[1], K, 2, 1, o1);
    o1 = recolour_byte(h0[2], h1[2], K, 0, 2, o1);
    o1 = recolour_byte(h0[2], h1[2], K, 1, 3, o1);
    o2 = recolour_byte(h0[2], h1[2], K, 2, 0, o2);
    o2 = recolour_byte(h0[3], h1[3], K, 0, 1, o2);
    o2 = recolour_byte(h0[3], h1[3], K, 1, 2, o2);
    o2 = recolour_byte(h0[3], h1[3], K, 2, 3, o2);
    u32x3 o;
    o.x = o0; o.y = o1; o.z = o2;
    return o;
}

// Recolours units [0, cnt) of a chunk: loads from rs, stores to ws (both over the chunk's bytes).
template <int COPIES, int UNROLL>
__device__ void p2_chunk(const P2Lds<COPIES>& T, const RecolourConsts& K, __amdgpu_buffer_rsrc_t rs,
                         __amdgpu_buffer_rsrc_t ws, int cnt, int tid, int nthreads) {
    const uint32_t roff = (uint32_t)((tid & 63) & (COPIES - 1)) << 3;
    const int stride = nthreads * UNROLL;
    u32x3 cur[UNROLL];
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (int lb = tid; lb < cnt; lb += stride) {
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j)
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb + stride + j * nthreads), 0, kLoadStream);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) p2_densities(T, roff, K, px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            __builtin_amdgcn_raw_buffer_store_b96(recolour_unit(h0, h1, K), ws, 12 * (lb + j * nthreads), 0, kStoreStream);
        }
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) cur[j] = nxt[j];
    }
}

// Grid-stride form of pass 2 (tiles of nthreads * UNROLL units, workgroup b takes tiles b,
// b + gridDim.x, ...).
template <int COPIES, int UNROLL>
__device__ void p2_tiles(const P2Lds<COPIES>& T, const RecolourConsts& K, const uint8_t* src, uint8_t* out,
                         int64_t n_units, int tid, int nthreads) {
    const uint32_t roff = (uint32_t)((tid & 63) & (COPIES - 1)) << 3;
    const int64_t tu = (int64_t)nthreads * UNROLL;
    const int64_t n_tiles = (n_units + tu - 1) / tu;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    auto tile_rs = [&](const uint8_t* base, int64_t tt) {   // one descriptor from selected fields
        const bool in = tt < n_tiles;
        return chunk_rsrc(base, in ? tt * tu : 0, in ? min(tu, n_units - tt * tu) : 0);
    };
    const __amdgpu_buffer_rsrc_t rs0 = tile_rs(src, t);
    u32x3 cur[UNROLL];
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs0, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (; t < n_tiles; t += gridDim.x) {
        const __amdgpu_buffer_rsrc_t rn = tile_rs(src, t + gridDim.x);   // empty past the end
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * nthreads), 0, kLoadStream);
        const __amdgpu_buffer_rsrc_t ws = tile_rs(out, t);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) p2_densities(T, roff, K, px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            __builtin_amdgcn_raw_buffer_store_b96(recolour_unit(h0, h1, K), ws, 12 * (tid + j * nthreads), 0, kStoreStream);
        }
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) cur[j] = nxt[j];
    }
}

// Tail pixels recoloured by one thread.
template <int COPIES>
__device__ void p2_tail(const P2Lds<COPIES>& T, const RecolourConsts& K, const uint8_t* src, uint8_t* out, int n) {
    const uint32_t roff = (uint32_t)((threadIdx.x & 63) & (COPIES - 1)) << 3;
    for (int i = 0; i < n; ++i) {
        float h0, h1;
        p2_densities(T, roff, K, src[3 * i], src[3 * i + 1], src[3 * i + 2], h0, h1);
        for (int c = 0; c < 3; ++c) out[3 * i + c] = (uint8_t)recolour_byte(h0, h1, K, c, 0, 0u);
    }
}

// ================================================================================== pass 1 + densities

// Pass 1 that also writes the FP32 densities of every pixel (Eq. 2, planar [2][n_px]): the same
// histogram as p1f_tiles, plus, per unit, four densities per stain from the FP32 pass-2 tables T
// (p2_densities, the arithmetic of the recolour pass), stored as one 16-byte write per stain plane.
// The planes are addressed through buffer resources (plane 1 starts at h + n_px, which is 16-byte
// aligned only when n_px is a multiple of 4; buffer stores need 4-byte alignment only).
template <bool WIDE, int UNROLL, bool U16>
__device__ void p1f_tiles_dens(P1FLds<WIDE>& S, const P2Lds<1>& T, const RecolourConsts& K, const P1Params& pp,
                               const uint8_t* src, int64_t n_units, float* h, int64_t n_px, int tid, int nthreads,
                               int64_t scatter, int64_t step) {
    const P1FLane L = p1f_lane<WIDE>(tid, pp.white_sum);
    const int64_t tu = (int64_t)nthreads * UNROLL;
    const int64_t n_tiles = (n_units + tu - 1) / tu;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    int64_t ph = (t * scatter) % n_tiles;
    auto tile_rs = [&](int64_t tt, int64_t tile) {
        const bool in = tt < n_tiles;
        return chunk_rsrc(src, in ? tile * tu : 0, in ? min(tu, n_units - tile * tu) : 0);
    };
    // plane descriptors over whole units of this tile: 16 bytes per unit and stain
    auto plane_rs = [&](const float* base, int64_t tile) {
        const uint64_t addr = reinterpret_cast<uint64_t>(base) + 16 * (uint64_t)(tile * tu);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
        const int nb = __builtin_amdgcn_readfirstlane((int)(16 * min(tu, n_units - tile * tu)));
        return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, nb, kBufDword3);
    };
    __amdgpu_buffer_rsrc_t rs = tile_rs(t, ph);
    P1FPend P = p1f_pend();
    u32x3 cur[UNROLL];
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (; t < n_tiles; t += gridDim.x) {
        int64_t pn = ph + step;
        if (pn >= n_tiles) pn -= n_tiles;
        const __amdgpu_buffer_rsrc_t rn = tile_rs(t + gridDim.x, pn);
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * nthreads), 0, kLoadStream);
        const int cnt = (int)min(tu, n_units - ph * tu);
        p1f_units<WIDE, UNROLL, U16>(S, pp, L, cur, tid, cnt, nthreads, P);
        const __amdgpu_buffer_rsrc_t w0 = plane_rs(h, ph), w1 = plane_rs(h + n_px, ph);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) p2_densities(T, 0u, K, px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            const int off = 16 * (tid + j * nthreads);   // past the tile's units the stores are dropped
            u32x4 v0, v1;
            v0.x = __float_as_uint(h0[0]); v0.y = __float_as_uint(h0[1]); v0.z = __float_as_uint(h0[2]); v0.w = __float_as_uint(h0[3]);
            v1.x = __float_as_uint(h1[0]); v1.y = __float_as_uint(h1[1]); v1.z = __float_as_uint(h1[2]); v1.w = __float_as_uint(h1[3]);
            __builtin_amdgcn_raw_buffer_store_b128(v0, w0, off, 0, kStoreStream);
            __builtin_amdgcn_raw_buffer_store_b128(v1, w1, off, 0, kStoreStream);
        }
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) cur[j] = nxt[j];
        ph = pn;
    }
    p1f_flush<WIDE, U16>(S, pp, L, P);
}

// Pass 1 with the densities for u = 16, from one set of fixed-point sums per unit: the candidate
// sums y_j of every pixel (p1f_unit_sums, all lanes) give both the histogram bins (as in pass 1, on
// the lanes whose unit holds a non-white pixel) and the densities h_j = max(0, y_j + kGuardUnits) /
// (2^16 * 256 / hist_hi_j) -- the table entries are within half a unit of their FP64 values, so a
// density is within 1.5 * hist_hi_j / 2^24 of the exact one.  Planes as in p1f_tiles_dens.
template <int UNROLL>
__device__ void p1f_tiles_dens16(P1FLds<true>& S, const P1Params& pp, const uint8_t* src, int64_t n_units, float* h,
                                 int64_t n_px, int tid, int nthreads, int64_t scatter, int64_t step) {
    const P1FLane L = p1f_lane<true>(tid, pp.white_sum);
    const int32_t thr = pp.white_sum > 0 ? pp.white_sum : 0x7FFFFFFF;
    const uint32_t nmask = p1f_nmask(16);
    const float c0 = (float)((double)pp.hist_hi[0] / 16777216.0), c1 = (float)((double)pp.hist_hi[1] / 16777216.0);
    const int64_t tu = (int64_t)nthreads * UNROLL;
    const int64_t n_tiles = (n_units + tu - 1) / tu;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return;
    int64_t ph = (t * scatter) % n_tiles;
    auto tile_rs = [&](int64_t tt, int64_t tile) {
        const bool in = tt < n_tiles;
        return chunk_rsrc(src, in ? tile * tu : 0, in ? min(tu, n_units - tile * tu) : 0);
    };
    auto plane_rs = [&](const float* base, int64_t tile) {
        const uint64_t addr = reinterpret_cast<uint64_t>(base) + 16 * (uint64_t)(tile * tu);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)addr);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
        const int nb = __builtin_amdgcn_readfirstlane((int)(16 * min(tu, n_units - tile * tu)));
        return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, nb, kBufDword3);
    };
    // one tile: the next tile's loads into nxt, then the densities and counts of cur's units
    auto tile_step = [&](const u32x3 (&cur)[UNROLL], u32x3 (&nxt)[UNROLL]) {
        int64_t pn = ph + step;
        if (pn >= n_tiles) pn -= n_tiles;
        const __amdgpu_buffer_rsrc_t rn = tile_rs(t + gridDim.x, pn);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rn, 12 * (tid + j * nthreads), 0, kLoadStream);
        const int cnt = (int)min(tu, n_units - ph * tu);
        const __amdgpu_buffer_rsrc_t w0 = plane_rs(h, ph), w1 = plane_rs(h + n_px, ph);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            const bool valid = tid + j * nthreads < cnt;
            const uint32_t X = cur[j].x, Y0 = cur[j].y, Z = cur[j].z;
            int32_t sum[4], y0[4], y1[4];
            p1f_white_sums(X, Y0, Z, sum);
            p1f_unit_sums(S, L, X, Y0, Z, y0, y1);
            u32x4 v0, v1;
            v0.x = __float_as_uint(fmaxf(0.0f, (float)(y0[0] + kGuardUnits) * c0));
            v0.y = __float_as_uint(fmaxf(0.0f, (float)(y0[1] + kGuardUnits) * c0));
            v0.z = __float_as_uint(fmaxf(0.0f, (float)(y0[2] + kGuardUnits) * c0));
            v0.w = __float_as_uint(fmaxf(0.0f, (float)(y0[3] + kGuardUnits) * c0));
            v1.x = __float_as_uint(fmaxf(0.0f, (float)(y1[0] + kGuardUnits) * c1));
            v1.y = __float_as_uint(fmaxf(0.0f, (float)(y1[1] + kGuardUnits) * c1));
            v1.z = __float_as_uint(fmaxf(0.0f, (float)(y1[2] + kGuardUnits) * c1));
            v1.w = __float_as_uint(fmaxf(0.0f, (float)(y1[3] + kGuardUnits) * c1));
            const int off = 16 * (tid + j * nthreads);   // past the tile's units the stores are dropped
            __builtin_amdgcn_raw_buffer_store_b128(v0, w0, off, 0, kStoreStream);
            __builtin_amdgcn_raw_buffer_store_b128(v1, w1, off, 0, kStoreStream);
            const bool tissue = valid && min(min(sum[0], sum[1]), min(sum[2], sum[3])) < thr;
            const uint64_t tl = __ballot(tissue);
            uint64_t nearm = 0;
            if (tissue) nearm = p1f_bins<true, true>(S, L, X, Y0, Z, y0, y1, nmask, tl);
            p1f_settle<true, true>(S, pp, L, X, Y0, Z, nearm, thr, nmask);
        }
        ph = pn;
        t += gridDim.x;
    };
    u32x3 ua[UNROLL], ub[UNROLL];   // two buffers taking turns, so no register copies between tiles
    const __amdgpu_buffer_rsrc_t rs = tile_rs(t, ph);
#pragma unroll
    for (int j = 0; j < UNROLL; ++j) ua[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, kLoadStream);
    for (;;) {
        tile_step(ua, ub);
        if (t >= n_tiles) break;
        tile_step(ub, ua);
        if (t >= n_tiles) break;
    }
}

}  // namespace spcn
