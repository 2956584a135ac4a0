// spcn_device.hpp -- device building blocks shared by the SPCN kernels (gfx950, wave64).
//
// Per-pixel density solve (Eq. 2 with W fixed).  With G = W^T W and b = W^T v - lambda/2, the
// unconstrained minimiser is f = G^-1 b and the one-stain minimisers are p_j = b_j / g_jj.  Because
// both stain vectors are non-negative, g01 >= 0, and p_0 = f_0 + (g01/g00) f_1 (likewise for stain
// 1).  The KKT conditions of the non-negative problem then give, in every region of the quadrant,
//     h_j = max(0, min(p_j, f_j)) = max(0, f_j + a_j * min(f_other, 0)),   a_0 = g01/g00, a_1 = g01/g11,
// which is what the kernels evaluate.  f and p are affine in the optical densities v, so each is a
// sum of three per-channel table entries indexed directly by the 8-bit intensities (Eq. 1 is folded
// into the tables, which are built in FP64 from the device-resident basis at kernel start).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spcn {

constexpr int kHistBins = 256;
constexpr double kLog2e = 1.4426950408889634073599246810019;
constexpr int kGuardUnits = 2;   // half-width of the FP64 recheck band, in table fixed-point units

// FP64 quantities derived once per launch from the basis and lambda.
struct Basis64 {
    double w[6];
    double g00, g01, g11, det;
    double q[2][3];       // rows of G^-1 W^T  (f = q v + fconst)
    double pc[2][3];      // W^T rows / g_jj   (p = pc v + pconst)
    double fconst[2], pconst[2];
    double a[2];          // a_0 = g01/g00, a_1 = g01/g11
    double half_lambda;
    int ok;               // Gram matrix positive definite and finite
};

// Plain sequential FP64 sums (no contraction) so the recheck path rounds like a textbook
// evaluation of the same expressions.  B.ok: finite, non-negative, Gram matrix positive definite.
__device__ inline void derive_basis(const float* __restrict__ w, float lambda, Basis64& B) {
#pragma clang fp contract(off)
    for (int i = 0; i < 6; ++i) B.w[i] = (double)w[i];
    const double* W = B.w;
    double g00 = W[0] * W[0]; g00 = g00 + W[1] * W[1]; g00 = g00 + W[2] * W[2];
    double g01 = W[0] * W[3]; g01 = g01 + W[1] * W[4]; g01 = g01 + W[2] * W[5];
    double g11 = W[3] * W[3]; g11 = g11 + W[4] * W[4]; g11 = g11 + W[5] * W[5];
    double det = g00 * g11 - g01 * g01;
    B.g00 = g00; B.g01 = g01; B.g11 = g11; B.det = det;
    bool finite = true, nonneg = true;
    for (int i = 0; i < 6; ++i) {
        finite = finite && (W[i] == W[i]) && (W[i] - W[i] == 0.0);
        nonneg = nonneg && W[i] >= 0.0;
    }
    // Eq. 2 constrains W >= 0, and the closed form below needs g01 >= 0, which W >= 0 gives: a basis
    // with a negative entry is outside the method and is refused like a singular one
    B.ok = finite && nonneg && g00 > 0.0 && g11 > 0.0 && det > 1e-12 * g00 * g11;
    double id = B.ok ? 1.0 / det : 0.0;
    double ig00 = B.ok ? 1.0 / g00 : 0.0, ig11 = B.ok ? 1.0 / g11 : 0.0;
    B.half_lambda = 0.5 * (double)lambda;
    for (int c = 0; c < 3; ++c) {
        B.q[0][c] = (g11 * W[c] - g01 * W[c + 3]) * id;
        B.q[1][c] = (g00 * W[c + 3] - g01 * W[c]) * id;
        B.pc[0][c] = W[c] * ig00;
        B.pc[1][c] = W[c + 3] * ig11;
    }
    B.fconst[0] = -B.half_lambda * (g11 - g01) * id;
    B.fconst[1] = -B.half_lambda * (g00 - g01) * id;
    B.pconst[0] = -B.half_lambda * ig00;
    B.pconst[1] = -B.half_lambda * ig11;
    B.a[0] = g01 * ig00;
    B.a[1] = g01 * ig11;
}

// Eq. (1) in FP64 for an 8-bit intensity: log(i0 / max(k, 1)), clamped at 0.
__device__ inline double od_u8(double i0, int k) {
    double v = log(i0 / (double)(k < 1 ? 1 : k));
    return v > 0.0 ? v : 0.0;
}

// FP64 densities of one pixel from its FP64 optical densities (recheck path of pass 1).
__device__ inline void solve64(const Basis64& B, double v0, double v1, double v2, double& h0, double& h1) {
#pragma clang fp contract(off)
    const double* W = B.w;
    double b0 = W[0] * v0; b0 = b0 + W[1] * v1; b0 = b0 + W[2] * v2; b0 = b0 - B.half_lambda;
    double b1 = W[3] * v0; b1 = b1 + W[4] * v1; b1 = b1 + W[5] * v2; b1 = b1 - B.half_lambda;
    double f0 = (B.g11 * b0 - B.g01 * b1) / B.det;
    double f1 = (B.g00 * b1 - B.g01 * b0) / B.det;
    double p0 = b0 / B.g00, p1 = b1 / B.g11;
    double t0 = p0 < f0 ? p0 : f0, t1 = p1 < f1 ? p1 : f1;
    h0 = t0 > 0.0 ? t0 : 0.0;
    h1 = t1 > 0.0 ? t1 : 0.0;
    if (!B.ok) { h0 = 0.0; h1 = 0.0; }
}

// Fixed-point resolution for the exact pass-1 tables: the largest u <= 20 such that any sum of
// three entries (plus rounding and the guard offset) stays below 2^30 in magnitude.
__device__ inline int table_shift(const Basis64& B, const float i0[3], const float hist_hi[2]) {
    double S = 0.0;
    for (int j = 0; j < 2; ++j) {
        double sigma = 256.0 / (double)hist_hi[j];
        double s = fmax(fabs(B.pconst[j]), fabs(B.fconst[j]));
        for (int c = 0; c < 3; ++c) s += fmax(fabs(B.pc[j][c]), fabs(B.q[j][c])) * od_u8((double)i0[c], 1);
        S = fmax(S, s * sigma);
    }
    if (!(S > 1e-30)) return 20;
    int u = ilogb(1073741824.0 / (S + 1.0));
    return u > 20 ? 20 : (u < 0 ? 0 : u);
}

// Histogram range of one stain: a device-resident value when one is given (for example the range
// spcn_estimate_basis derives from its sample percentile), else the host parameter.  A device value
// is rounded up to a power of two and clamped to [2^-8, 2^8]; one that is not finite and positive
// falls back to the host value.
__device__ inline float resolve_range(const float* dev, float host) {
    if (!dev) return host;
    const float v = *dev;
    if (!(v > 0.0f) || !(v <= 3.0e38f)) return host;
    int e;
    const float m = frexpf(v, &e);                   // v = m 2^e, m in [0.5, 1)
    const float r = m == 0.5f ? v : ldexpf(1.0f, e);
    return fminf(fmaxf(r, 0.00390625f), 256.0f);
}

// Histogram range derived from a sample percentile P: the power of two 2^ceil(log2(2 P)), clamped
// to [2^-4, 2^6], so that a percentile of the whole image near P falls in bins 64..127.
__device__ inline float range_for_percentile(double P) {
    const double v = 2.0 * P;
    if (!(v > 0.0625)) return 0.0625f;
    if (!(v < 64.0)) return 64.0f;
    int e;
    const double m = frexp(v, &e);                   // v = m 2^e, m in [0.5, 1)
    return (float)(m == 0.5 ? v : ldexp(1.0, e));
}

// Histogram percentile (Eq. 3) of one stain from inclusive cumulative counts, evaluated by the
// thread that owns the crossing bin k* = min{k : C_k >= q n}:
//     P = width * (k* + (q n - C_{k*-1}) / c_{k*}).
// Returns true on the owning thread.
__device__ inline bool percentile_owner(const uint64_t* cum, int k, double q, double hist_hi, double& P) {
#pragma clang fp contract(off)
    uint64_t n = cum[kHistBins - 1];
    if (n == 0) return false;
    double r = q * (double)n;
    uint64_t C = cum[k], Cp = k ? cum[k - 1] : 0;
    if (!((double)C >= r) || (k && !((double)Cp < r))) return false;
    double width = hist_hi / (double)kHistBins;
    P = width * ((double)k + (r - (double)Cp) / (double)(C - Cp));
    return true;
}

}  // namespace spcn
