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
// reads copy l % COPIES, so the 8 lanes that share an LDS cycle for 16-byte reads hit distinct banks
// whatever their intensities.  The histogram keeps one private column per lane % COLS, so lanes that
// share an LDS cycle never increment the same word.
#pragma once

#include "spcn_device.hpp"
#include "../../include/spcn.h"

namespace spcn {

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
constexpr int kBufDword3 = 0x00020000;   // raw (untyped) buffer, gfx9-family descriptor word 3

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
};

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
        const bool near = ((x0 & fmask) < 2 * kGuardUnits) | ((x1 & fmask) < 2 * kGuardUnits);
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
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, 0);
    for (int lb = tid; lb < cnt; lb += stride) {
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j)   // prefetch; past the chunk the loads return zeros
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb + stride + j * nthreads), 0, 0);
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
                    const bool near = ((x0[q] & fmask) < 2 * kGuardUnits) | ((x1[q] & fmask) < 2 * kGuardUnits);
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
        if (((x0 & fmask) < 2 * kGuardUnits) | ((x1 & fmask) < 2 * kGuardUnits)) {
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

// Scale of Eq. (3): no tissue or a percentile in bin 0 keeps the density unscaled.
__device__ inline double stain_scale(double scale_tgt, double P, int fl) {
    if ((fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0)) || !(P > 0.0)) return 1.0;
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
    for (int j = 0; j < UNROLL; ++j) cur[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (tid + j * nthreads), 0, 0);
    for (int lb = tid; lb < cnt; lb += stride) {
        u32x3 nxt[UNROLL];
#pragma unroll
        for (int j = 0; j < UNROLL; ++j)
            nxt[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb + stride + j * nthreads), 0, 0);
#pragma unroll
        for (int j = 0; j < UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(cur[j], px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) p2_densities(T, roff, K, px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            __builtin_amdgcn_raw_buffer_store_b96(recolour_unit(h0, h1, K), ws, 12 * (lb + j * nthreads), 0, 0);
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

}  // namespace spcn
