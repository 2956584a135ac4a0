// spcn_u8.hip -- fused SPCN normalisation of one uint8 RGB image on gfx950.
//
// Two streaming passes over the interleaved 3-byte pixels (the method's Eqs. 1-4, Sec. 2.1; the
// non-white percentile of Sec. 3.1 item 2):
//   pass 1  (k_pass1)  reads 3 B/px: Eq. 1 + Eq. 2 per non-white pixel, 2 x 256-bin histogram of
//                      the densities (optionally also writes FP32 densities, 8 B/px);
//   pass 2  (k_pass2)  percentile of Eq. 3 from the histogram (every workgroup recomputes it in its
//                      prologue, so there is no separate finalisation launch), then re-reads 3 B/px,
//                      re-solves, scales, recolours (Eq. 3), applies Eq. 4 and writes 3 B/px.
//
// Memory layout: a thread handles 4-pixel units (12 bytes = 3 dwords, one dwordx3 load), so a
// wavefront reads 768 contiguous bytes per load instruction.  Workgroups own contiguous chunks.
//
// Exact histogram counts: pass 1 evaluates the two candidate values p_j and f_j of each stain as
// sums of three int32 fixed-point table entries (2^-u bin units, u <= 20).  Integer sums are exact,
// so each candidate is within 1.5 units of its exact value; a pixel whose value is within
// kGuardUnits of a bin edge is re-solved in FP64 (a rare, divergent path) before it is binned.
// Bin decisions therefore equal those of exact arithmetic (and of an FP64 evaluation).
#include "spcn_internal.h"
#include "spcn_device.hpp"

namespace spcn {

namespace {

constexpr int P1_THREADS = 1024;   // one workgroup per CU: the lane-private histogram takes 128 KB
constexpr int P1_UNROLL = 4;       // 4-pixel units per thread per iteration
constexpr int P2_THREADS = 256;
constexpr int P2_UNROLL = 4;
constexpr int HIST_WORDS = 2 * kHistBins * 64;   // [stain][bin][lane] uint32

struct P1Args {
    const uint8_t* src;
    int64_t n_px;
    const float* w;
    float i0[3];
    float lambda;
    int32_t white_sum;
    float hist_hi[2];
    uint64_t* hist;      // global [2][256]
    float* h_out;        // optional planar FP32 densities
};

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
    double q;
    const uint64_t* hist;
    float* p99_out;
    float* scale_out;
    int32_t* flags_out;
};

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
constexpr int kBufDword3 = 0x00020000;   // raw (untyped) buffer, gfx9-family descriptor word 3

// Buffer resource over one workgroup's chunk of 4-pixel units: 32-bit offsets, and the hardware
// range check returns zeros for loads past the end and drops stores past the end.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void* base, int64_t unit0, int64_t units) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(static_cast<const uint8_t*>(base)) + 12 * unit0,
                                             0, (int)(12 * units), kBufDword3);
}

__device__ __forceinline__ void bytes_of_unit(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t px[4][3]) {
    px[0][0] = d0 & 0xFF;         px[0][1] = (d0 >> 8) & 0xFF;  px[0][2] = (d0 >> 16) & 0xFF;
    px[1][0] = d0 >> 24;          px[1][1] = d1 & 0xFF;         px[1][2] = (d1 >> 8) & 0xFF;
    px[2][0] = (d1 >> 16) & 0xFF; px[2][1] = d1 >> 24;          px[2][2] = d2 & 0xFF;
    px[3][0] = (d2 >> 8) & 0xFF;  px[3][1] = (d2 >> 16) & 0xFF; px[3][2] = d2 >> 24;
}

// ----------------------------------------------------------------------------- pass 1

struct P1Shared {
    int4 tab[3 * kHistBins];       // (p0, f0, p1, f1) fixed point, per channel and intensity
    float2 ftab[3 * kHistBins];    // (f0, f1) FP32 density units, for the optional density output
    double od[3 * kHistBins];      // FP64 Eq. 1, for the recheck path
    Basis64 B;
    int shift;
    uint32_t hist[HIST_WORDS];     // 128 KB, lane-private columns: no two lanes of a wave collide
};

template <bool STORE_H>
__global__ __launch_bounds__(P1_THREADS) void k_pass1(const P1Args a) {
    __shared__ P1Shared S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;

    for (int i = tid; i < HIST_WORDS; i += P1_THREADS) S.hist[i] = 0u;
    if (tid == 0) {
        derive_basis(a.w, a.lambda, S.B);
        S.shift = table_shift(S.B, a.i0, a.hist_hi);
    }
    __syncthreads();
    const int u = S.shift;
    if (tid < kHistBins) {
        const int k = tid;
        for (int c = 0; c < 3; ++c) {
            double od = S.B.ok ? od_u8((double)a.i0[c], k) : 0.0;
            S.od[c * kHistBins + k] = od;
            int4 e;
            int32_t ent[4];
            for (int j = 0; j < 2; ++j) {
                double sig = ldexp(256.0 / (double)a.hist_hi[j], u);
                double pv = S.B.pc[j][c] * od + (c == 0 ? S.B.pconst[j] : 0.0);
                double fv = S.B.q[j][c] * od + (c == 0 ? S.B.fconst[j] : 0.0);
                ent[2 * j] = __double2int_rn(pv * sig) + (c == 0 ? kGuardUnits : 0);
                ent[2 * j + 1] = __double2int_rn(fv * sig) + (c == 0 ? kGuardUnits : 0);
            }
            e.x = ent[0]; e.y = ent[1]; e.z = ent[2]; e.w = ent[3];
            S.tab[c * kHistBins + k] = e;
            if (STORE_H) {
                float2 f;
                f.x = (float)(S.B.q[0][c] * od + (c == 0 ? S.B.fconst[0] : 0.0));
                f.y = (float)(S.B.q[1][c] * od + (c == 0 ? S.B.fconst[1] : 0.0));
                S.ftab[c * kHistBins + k] = f;
            }
        }
    }
    __syncthreads();

    const int32_t thr = a.white_sum > 0 ? a.white_sum : 0x7FFFFFFF;
    const int32_t fmask = (1 << u) - 1;
    const float fa0 = (float)S.B.a[0], fa1 = (float)S.B.a[1];
    uint32_t* hist0 = S.hist + lane;
    uint32_t* hist1 = S.hist + kHistBins * 64 + lane;

    const double sg0 = 256.0 / (double)a.hist_hi[0], sg1 = 256.0 / (double)a.hist_hi[1];

    // Fixed-point candidates of one pixel: x_j = min(p_j, f_j) in 2^-u bin units (+ guard offset).
    auto fixed_bins = [&](uint32_t R, uint32_t G, uint32_t Bc, int32_t& x0, int32_t& x1) {
        int4 tr = S.tab[R], tg = S.tab[kHistBins + G], tb = S.tab[2 * kHistBins + Bc];
        x0 = min(tr.x + tg.x + tb.x, tr.y + tg.y + tb.y);
        x1 = min(tr.z + tg.z + tb.z, tr.w + tg.w + tb.w);
    };
    auto is_near = [&](int32_t x0, int32_t x1) {
        return ((x0 & fmask) < 2 * kGuardUnits) | ((x1 & fmask) < 2 * kGuardUnits);
    };
    auto count_fixed = [&](int32_t x0, int32_t x1) {
        int k0 = min(max(x0 >> u, 0), kHistBins - 1);
        int k1 = min(max(x1 >> u, 0), kHistBins - 1);
        atomicAdd(hist0 + (k0 << 6), 1u);
        atomicAdd(hist1 + (k1 << 6), 1u);
    };
    // Cold path: the pixel lies within kGuardUnits of a bin edge; decide its bins in FP64.
    auto count_fp64 = [&](uint32_t R, uint32_t G, uint32_t Bc) {
        double d0, d1;
        solve64(S.B, S.od[R], S.od[kHistBins + G], S.od[2 * kHistBins + Bc], d0, d1);
        double e0 = floor(d0 * sg0), e1 = floor(d1 * sg1);
        int k0 = e0 >= 255.0 ? 255 : (int)e0;
        int k1 = e1 >= 255.0 ? 255 : (int)e1;
        atomicAdd(hist0 + (k0 << 6), 1u);
        atomicAdd(hist1 + (k1 << 6), 1u);
    };
    // Densities in FP32 for the optional output.
    auto dens32 = [&](uint32_t R, uint32_t G, uint32_t Bc, float& h0, float& h1) {
        float2 r = S.ftab[R], g = S.ftab[kHistBins + G], b = S.ftab[2 * kHistBins + Bc];
        float f0 = r.x + g.x + b.x, f1 = r.y + g.y + b.y;
        h0 = fmaxf(0.0f, fmaf(fa0, fminf(f1, 0.0f), f0));   // tables are zero for a singular basis
        h1 = fmaxf(0.0f, fmaf(fa1, fminf(f0, 0.0f), f1));
    };
    // Full exact treatment of one pixel read from memory (cold re-check loop and the image tail):
    // only pixels that are near a bin edge are counted here when `only_near` is set.
    auto exact_pixel = [&](int64_t i, bool only_near) {
        const uint8_t* p = a.src + 3 * i;
        uint32_t R = p[0], G = p[1], Bc = p[2];
        if ((int32_t)(R + G + Bc) >= thr) return;
        int32_t x0, x1;
        fixed_bins(R, G, Bc, x0, x1);
        if (is_near(x0, x1)) count_fp64(R, G, Bc);
        else if (!only_near) count_fixed(x0, x1);
    };

    const int64_t n_units = a.n_px >> 2;
    const int64_t per = (n_units + gridDim.x - 1) / gridDim.x;
    const int64_t ubeg = min(n_units, (int64_t)blockIdx.x * per);
    const int cnt = (int)(min(n_units, ubeg + per) - ubeg);     // units of this workgroup
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.src, ubeg, cnt);

    for (int lb = tid; lb < cnt; lb += P1_THREADS * P1_UNROLL) {
        uint32_t px[P1_UNROLL][4][3];
        bool tis[P1_UNROLL][4];
        bool any_tissue = false;
#pragma unroll
        for (int j = 0; j < P1_UNROLL; ++j) {
            const int lu = lb + j * P1_THREADS;
            const u32x3 d = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * lu, 0, 0);
            bytes_of_unit(d.x, d.y, d.z, px[j]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                tis[j][q] = lu < cnt && (int32_t)(px[j][q][0] + px[j][q][1] + px[j][q][2]) < thr;
                any_tissue |= tis[j][q];
            }
        }
        bool any_near = false;
        if (STORE_H || any_tissue) {
#pragma unroll
            for (int j = 0; j < P1_UNROLL; ++j) {
                const int lu = lb + j * P1_THREADS;
                float h0[4], h1[4];
                int32_t x0[4], x1[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (STORE_H) dens32(px[j][q][0], px[j][q][1], px[j][q][2], h0[q], h1[q]);
                    fixed_bins(px[j][q][0], px[j][q][1], px[j][q][2], x0[q], x1[q]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (tis[j][q]) {
                        const bool near = is_near(x0[q], x1[q]);
                        any_near |= near;
                        if (!near) count_fixed(x0[q], x1[q]);
                    }
                }
                if (STORE_H && lu < cnt) {
                    const int64_t un = ubeg + lu;
                    *reinterpret_cast<float4*>(a.h_out + 4 * un) = make_float4(h0[0], h0[1], h0[2], h0[3]);
                    float* h1p = a.h_out + a.n_px + 4 * un;
                    if ((a.n_px & 3) == 0) {
                        *reinterpret_cast<float4*>(h1p) = make_float4(h1[0], h1[1], h1[2], h1[3]);
                    } else {
                        h1p[0] = h1[0]; h1p[1] = h1[1]; h1p[2] = h1[2]; h1p[3] = h1[3];
                    }
                }
            }
        }
        if (any_near) {   // rare: re-read this thread's pixels and settle the near-edge ones in FP64
#pragma unroll 1
            for (int b = 0; b < 4 * P1_UNROLL; ++b) {
                const int lu = lb + (b >> 2) * P1_THREADS;
                if (lu < cnt) exact_pixel(4 * (ubeg + lu) + (b & 3), true);
            }
        }
    }
    // the last n_px % 4 pixels
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        for (int64_t i = n_units * 4; i < a.n_px; ++i) {
            exact_pixel(i, false);
            if (STORE_H) {
                const uint8_t* p = a.src + 3 * i;
                float h0, h1;
                dens32(p[0], p[1], p[2], h0, h1);
                a.h_out[i] = h0; a.h_out[a.n_px + i] = h1;
            }
        }
    }
    __syncthreads();

    // merge the lane-private columns and publish this workgroup's counts
    if (tid < 2 * kHistBins) {
        const uint32_t* row = S.hist + tid * 64;
        uint32_t sum = 0;
        for (int l = 0; l < 64; ++l) sum += row[(l + tid) & 63];   // rotated: no bank conflicts
        if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(a.hist) + tid, (unsigned long long)sum);
    }
}

// ----------------------------------------------------------------------------- finalisation

struct FinalShared {
    uint64_t cum[2][kHistBins];
    double P[2];
    int kstar[2];
};

// Eq. (3) percentile of both stains from the global histogram, computed by a 256-thread block.
// Afterwards F.P[j] and F.kstar[j] (-1: no tissue) are valid on every thread.
__device__ void block_percentiles(const uint64_t* __restrict__ hist, double q, const float hist_hi[2],
                                  FinalShared& F) {
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

// Flags and scale of one stain from its percentile (Eq. 3): no tissue or a percentile in bin 0
// keeps the density unscaled.
__device__ inline int stain_flags(const FinalShared& F, int j, bool basis_ok) {
    int fl = 0;
    if (F.kstar[j] < 0) fl |= SPCN_FLAG_NO_TISSUE;
    if (F.kstar[j] == kHistBins - 1) fl |= SPCN_FLAG_RANGE;
    if (F.kstar[j] == 0) fl |= SPCN_FLAG_BIN0;
    if (!basis_ok) fl |= SPCN_FLAG_BASIS;
    return fl;
}

__device__ inline double stain_scale(double scale_tgt, double P, int fl) {
    if ((fl & (SPCN_FLAG_NO_TISSUE | SPCN_FLAG_BIN0)) || !(P > 0.0)) return 1.0;
    return scale_tgt / P;
}

__global__ __launch_bounds__(256) void k_finalize(const uint64_t* hist, double q, float hh0, float hh1,
                                                  const float* w, float lambda, float* p99_out,
                                                  int32_t* flags_out) {
    __shared__ FinalShared F;
    __shared__ int basis_ok;
    const float hh[2] = {hh0, hh1};
    if (threadIdx.x == 0) { Basis64 B; derive_basis(w, lambda, B); basis_ok = B.ok; }
    block_percentiles(hist, q, hh, F);
    if (threadIdx.x < 2) {
        const int j = threadIdx.x;
        if (p99_out) p99_out[j] = (float)F.P[j];
        if (flags_out) flags_out[j] = stain_flags(F, j, basis_ok);
    }
}

__global__ void k_zero_u64(uint64_t* p, int n) {
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) p[i] = 0;
}

// ----------------------------------------------------------------------------- pass 2

struct P2Shared {
    float2 ftab[3 * kHistBins];
    FinalShared F;
    Basis64 B;
    float M[3][2];      // log2(e) * W_tgt[c,j] * s_j
    float L[3];         // log2(i0_out[c])
};

__device__ __forceinline__ uint32_t recolour(float h0, float h1, const float (&M)[3][2], const float (&L)[3],
                                             int c, uint32_t sel, uint32_t acc) {
    float z = fmaf(-M[c][0], h0, L[c]);
    z = fmaf(-M[c][1], h1, z);
    return __builtin_amdgcn_cvt_pk_u8_f32(__builtin_amdgcn_exp2f(z), sel, acc);
}

__global__ __launch_bounds__(P2_THREADS) void k_pass2(const P2Args a) {
    __shared__ P2Shared S;
    const int tid = threadIdx.x;
    if (tid == 0) derive_basis(a.w_src, a.lambda, S.B);
    __syncthreads();
    {
        const int k = tid;   // P2_THREADS == 256 == kHistBins
        for (int c = 0; c < 3; ++c) {
            double od = S.B.ok ? od_u8((double)a.i0[c], k) : 0.0;
            float2 f;
            f.x = (float)(S.B.q[0][c] * od + (c == 0 ? S.B.fconst[0] : 0.0));
            f.y = (float)(S.B.q[1][c] * od + (c == 0 ? S.B.fconst[1] : 0.0));
            S.ftab[c * kHistBins + k] = f;
        }
    }
    block_percentiles(a.hist, a.q, a.hist_hi, S.F);
    if (tid == 0) {
        double s[2];
        int fl[2];
        for (int j = 0; j < 2; ++j) {
            fl[j] = stain_flags(S.F, j, S.B.ok);
            s[j] = stain_scale((double)a.scale_tgt[j], S.F.P[j], fl[j]);
        }
        for (int c = 0; c < 3; ++c) {
            for (int j = 0; j < 2; ++j) S.M[c][j] = (float)(kLog2e * (double)a.w_tgt[c + 3 * j] * s[j]);
            S.L[c] = (float)log2((double)a.i0_out[c]);
        }
        if (blockIdx.x == 0) {
            for (int j = 0; j < 2; ++j) {
                if (a.p99_out) a.p99_out[j] = (float)S.F.P[j];
                if (a.scale_out) a.scale_out[j] = (float)s[j];
                if (a.flags_out) a.flags_out[j] = fl[j];
            }
        }
    }
    __syncthreads();

    float M[3][2], L[3];
    for (int c = 0; c < 3; ++c) {
        M[c][0] = S.M[c][0]; M[c][1] = S.M[c][1]; L[c] = S.L[c];
    }
    const float fa0 = (float)S.B.a[0], fa1 = (float)S.B.a[1];

    auto densities = [&](uint32_t R, uint32_t G, uint32_t Bc, float& h0, float& h1) {
        float2 r = S.ftab[R], g = S.ftab[kHistBins + G], b = S.ftab[2 * kHistBins + Bc];
        float f0 = r.x + g.x + b.x, f1 = r.y + g.y + b.y;
        h0 = fmaxf(0.0f, fmaf(fa0, fminf(f1, 0.0f), f0));   // tables are zero for a singular basis
        h1 = fmaxf(0.0f, fmaf(fa1, fminf(f0, 0.0f), f1));
    };

    const int64_t n_units = a.n_px >> 2;
    const int64_t per = (n_units + gridDim.x - 1) / gridDim.x;
    const int64_t ubeg = min(n_units, (int64_t)blockIdx.x * per);
    const int cnt = (int)(min(n_units, ubeg + per) - ubeg);
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.src, ubeg, cnt);
    const __amdgpu_buffer_rsrc_t ws = chunk_rsrc(a.out, ubeg, cnt);

    for (int lb = tid; lb < cnt; lb += P2_THREADS * P2_UNROLL) {
        u32x3 d[P2_UNROLL];
#pragma unroll
        for (int j = 0; j < P2_UNROLL; ++j)
            d[j] = __builtin_amdgcn_raw_buffer_load_b96(rs, 12 * (lb + j * P2_THREADS), 0, 0);
#pragma unroll
        for (int j = 0; j < P2_UNROLL; ++j) {
            uint32_t px[4][3];
            bytes_of_unit(d[j].x, d[j].y, d[j].z, px);
            float h0[4], h1[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) densities(px[q][0], px[q][1], px[q][2], h0[q], h1[q]);
            u32x3 o;
            uint32_t o0 = 0, o1 = 0, o2 = 0;
            o0 = recolour(h0[0], h1[0], M, L, 0, 0, o0);
            o0 = recolour(h0[0], h1[0], M, L, 1, 1, o0);
            o0 = recolour(h0[0], h1[0], M, L, 2, 2, o0);
            o0 = recolour(h0[1], h1[1], M, L, 0, 3, o0);
            o1 = recolour(h0[1], h1[1], M, L, 1, 0, o1);
            o1 = recolour(h0[1], h1[1], M, L, 2, 1, o1);
            o1 = recolour(h0[2], h1[2], M, L, 0, 2, o1);
            o1 = recolour(h0[2], h1[2], M, L, 1, 3, o1);
            o2 = recolour(h0[2], h1[2], M, L, 2, 0, o2);
            o2 = recolour(h0[3], h1[3], M, L, 0, 1, o2);
            o2 = recolour(h0[3], h1[3], M, L, 1, 2, o2);
            o2 = recolour(h0[3], h1[3], M, L, 2, 3, o2);
            o.x = o0; o.y = o1; o.z = o2;
            __builtin_amdgcn_raw_buffer_store_b96(o, ws, 12 * (lb + j * P2_THREADS), 0, 0);   // past-end: dropped
        }
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        for (int64_t i = n_units * 4; i < a.n_px; ++i) {
            const uint8_t* p = a.src + 3 * i;
            float h0, h1;
            densities(p[0], p[1], p[2], h0, h1);
            for (int c = 0; c < 3; ++c) a.out[3 * i + c] = (uint8_t)recolour(h0, h1, M, L, c, 0, 0u);
        }
    }
}

}  // namespace

// ----------------------------------------------------------------------------- launchers

size_t u8_workspace_bytes() { return 2 * kHistBins * sizeof(uint64_t); }

static int p1_grid(int64_t n_px, const DevInfo& dev) {
    int64_t units = n_px >> 2;
    int64_t want = (units + (int64_t)P1_THREADS * P1_UNROLL - 1) / ((int64_t)P1_THREADS * P1_UNROLL);
    if (want < 1) want = 1;
    return (int)(want < dev.cus ? want : dev.cus);
}

static int p2_grid(int64_t n_px, const DevInfo& dev) {
    int64_t units = n_px >> 2;
    int64_t want = (units + (int64_t)P2_THREADS * P2_UNROLL - 1) / ((int64_t)P2_THREADS * P2_UNROLL);
    if (want < 1) want = 1;
    int64_t cap = (int64_t)dev.cus * 8;
    return (int)(want < cap ? want : cap);
}

hipError_t launch_densities(const uint8_t* img, int64_t n_px, const float* w, const ParamsK& pk,
                            float* h_out, uint64_t* hist, float* p99_out, int32_t* flags_out,
                            const DevInfo& dev, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(256), 0, s, hist, 2 * kHistBins);
    P1Args a{};
    a.src = img; a.n_px = n_px; a.w = w;
    for (int c = 0; c < 3; ++c) a.i0[c] = pk.i0[c];
    a.lambda = pk.lambda; a.white_sum = pk.white_sum;
    a.hist_hi[0] = pk.hist_hi[0]; a.hist_hi[1] = pk.hist_hi[1];
    a.hist = hist; a.h_out = h_out;
    const int g = p1_grid(n_px, dev);
    if (h_out) hipLaunchKernelGGL(k_pass1<true>, dim3(g), dim3(P1_THREADS), 0, s, a);
    else hipLaunchKernelGGL(k_pass1<false>, dim3(g), dim3(P1_THREADS), 0, s, a);
    if (p99_out || flags_out)
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, hist, pk.q64, pk.hist_hi[0], pk.hist_hi[1],
                           w, pk.lambda, p99_out, flags_out);
    return hipGetLastError();
}

hipError_t launch_recolor(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                          const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                          uint8_t* out, const uint64_t* hist, float* p99_out, float* scale_out,
                          int32_t* flags_out, const DevInfo& dev, hipStream_t s) {
    P2Args b{};
    b.src = src; b.out = out; b.n_px = n_px; b.w_src = w_src; b.w_tgt = w_tgt; b.scale_tgt = scale_tgt;
    for (int c = 0; c < 3; ++c) { b.i0[c] = pk.i0[c]; b.i0_out[c] = i0_out[c]; }
    b.lambda = pk.lambda; b.hist_hi[0] = pk.hist_hi[0]; b.hist_hi[1] = pk.hist_hi[1];
    b.q = pk.q64; b.hist = hist;
    b.p99_out = p99_out; b.scale_out = scale_out; b.flags_out = flags_out;
    hipLaunchKernelGGL(k_pass2, dim3(p2_grid(n_px, dev)), dim3(P2_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_normalize(const uint8_t* src, int64_t n_px, const float* w_src, const float* w_tgt,
                            const float* scale_tgt, const float i0_out[3], const ParamsK& pk,
                            uint8_t* out, uint64_t* hist, float* p99_out, float* scale_out,
                            int32_t* flags_out, const DevInfo& dev, hipStream_t s) {
    hipError_t e = launch_densities(src, n_px, w_src, pk, nullptr, hist, nullptr, nullptr, dev, s);
    if (e != hipSuccess) return e;
    return launch_recolor(src, n_px, w_src, w_tgt, scale_tgt, i0_out, pk, out, hist, p99_out, scale_out,
                          flags_out, dev, s);
}

}  // namespace spcn
