"""FP64 CPU oracle for SPCN -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this package.
The product (paper_1901_03088_amd) never imports it, and the two share no code.

Thin numpy/ctypes wrapper over liboracle.so (spcn_oracle.c).  All scalars handed to the library in
FP32 (W, lambda, i0, scales, percentile) are widened exactly to float64 here, so the oracle sees
the same numbers the GPU path receives.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, NO_TISSUE, RANGE, BIN0, RANGE_RETRY = 0, 1, 2, 4, 256

_d = C.POINTER(C.c_double)
_u8 = C.POINTER(C.c_uint8)
_u64 = C.POINTER(C.c_uint64)
_i64 = C.POINTER(C.c_int64)
_f = C.POINTER(C.c_float)
_i = C.POINTER(C.c_int)


def lib():
    global _LIB
    if _LIB is None:
        # SPCN_ORACLE_LIB: another build of the same source (the sanitizer test loads an instrumented one)
        path = os.environ.get("SPCN_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.orc_od_u8.restype = C.c_double; L.orc_od_u8.argtypes = [C.c_double, C.c_int]
        L.orc_od_f.restype = C.c_double; L.orc_od_f.argtypes = [C.c_double, C.c_double]
        L.orc_solve_pixel.restype = C.c_int; L.orc_solve_pixel.argtypes = [_d, C.c_double, _d, _d]
        L.orc_is_tissue_u8.restype = C.c_int; L.orc_is_tissue_u8.argtypes = [_u8, C.c_int]
        L.orc_is_tissue_f32.restype = C.c_int
        L.orc_is_tissue_f32.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int]
        L.orc_densities_u8.restype = None
        L.orc_densities_u8.argtypes = [_u8, C.c_int64, _d, _d, C.c_double, C.c_int, _d, _u8]
        L.orc_histogram.restype = None
        L.orc_histogram.argtypes = [_d, _u8, C.c_int64, _d, C.c_int, _u64]
        L.orc_percentile_hist.restype = C.c_int
        L.orc_percentile_hist.argtypes = [_u64, C.c_int, C.c_double, C.c_double, _d, _i]
        L.orc_settle_range.restype = C.c_int
        L.orc_settle_range.argtypes = [_d, _u8, C.c_int64, _d, C.c_int, C.c_double, _d]
        L.orc_percentile_exact.restype = C.c_int
        L.orc_percentile_exact.argtypes = [_d, _u8, C.c_int64, C.c_double, _d, _i64]
        L.orc_normalize_u8.restype = C.c_int
        L.orc_normalize_u8.argtypes = [_u8, C.c_int64, _d, _d, _d, _d, _d, C.c_double, C.c_int, C.c_double,
                                       _d, C.c_int, _u8, _d, _u64]
        L.orc_reconstruct_pixel.restype = None
        L.orc_reconstruct_pixel.argtypes = [_d, _d, _d, _d, _d]
        L.orc_splitmix64.restype = C.c_uint64; L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_sample_tissue.restype = C.c_int64
        L.orc_sample_tissue.argtypes = [_u8, C.c_int64, C.c_int, C.c_uint64, C.c_int64, C.c_int64, _i64]
        L.orc_recolor_u8.restype = None
        L.orc_recolor_u8.argtypes = [_u8, C.c_int64, _d, _d, _d, _d, _d, _d, C.c_double, C.c_int, _u8]
        L.orc_band_percentiles.restype = C.c_int
        L.orc_band_percentiles.argtypes = [_u8, C.c_int64, C.c_int64, _d, _d, C.c_double, C.c_int, C.c_double, _d,
                                           C.c_int, C.c_int64, _d, _i, _d]
        L.orc_sample_percentile.restype = C.c_int
        L.orc_sample_percentile.argtypes = [_u8, C.c_int64, _d, _d, C.c_double, C.c_int, C.c_uint64, C.c_int64,
                                            C.c_int64, C.c_double, _d, _i64]
        L.orc_exact_percentile_u8.restype = C.c_int
        L.orc_exact_percentile_u8.argtypes = [_u8, C.c_int64, _d, _d, C.c_double, C.c_int, C.c_double, _d, _i64]
        L.orc_estimate_i0.restype = C.c_int64
        L.orc_estimate_i0.argtypes = [_u8, C.c_int64, C.c_int, C.c_uint64, C.c_int64, C.c_int64, C.c_double, _d]
        L.orc_nmf_objective.restype = C.c_double
        L.orc_nmf_objective.argtypes = [_d, _d, C.c_int64, _d, C.c_double]
        L.orc_nmf.restype = None
        L.orc_nmf.argtypes = [_d, C.c_int64, C.c_double, C.c_int, _d, _d, C.c_double, _d]
        L.orc_stain_order_swap.restype = C.c_int; L.orc_stain_order_swap.argtypes = [_d]
        L.orc_forward_f32.restype = C.c_int
        L.orc_forward_f32.argtypes = [_d, C.c_int64, _d, _d, _d, _d, _d, C.c_double, C.c_int, C.c_double,
                                      _d, _d, _i64, _d]
        L.orc_backward_f32.restype = C.c_int
        L.orc_backward_f32.argtypes = [_d, C.c_int64, _d, _d, _d, _d, _d, C.c_double, C.c_int, C.c_double,
                                       _d, _i64, _d, _d, _d]
        L.orc_active_margin_f32.restype = None
        L.orc_active_margin_f32.argtypes = [_d, C.c_int64, _d, _d, C.c_double, _d]
        _LIB = L
    return _LIB


# ------------------------------------------------------------------ helpers

def _p(a, t):
    return a.ctypes.data_as(t)


def f32(x) -> np.ndarray:
    """Round to FP32 and widen back to float64: the values the GPU path receives."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def basis(W) -> np.ndarray:
    """3x2 matrix or 6-vector (column-major) -> contiguous float64 6-vector W[c + 3 j]."""
    W = np.asarray(W, dtype=np.float64)
    if W.shape == (3, 2):
        W = W.T.reshape(6)
    return np.ascontiguousarray(W.reshape(6))


def _vec(x, n):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (n,)))


def _img(img) -> np.ndarray:
    a = np.asarray(img)
    assert a.dtype == np.uint8 and a.shape[-1] == 3
    return np.ascontiguousarray(a.reshape(-1, 3))


# ------------------------------------------------------------------ Eq. (1)-(2)

def od_u8(i0, intensity) -> float:
    return lib().orc_od_u8(float(i0), int(intensity))


def od_f(i0, x) -> float:
    return lib().orc_od_f(float(i0), float(x))


def solve_pixel(W, lam, v):
    W = basis(W); v = _vec(v, 3); h = np.zeros(2)
    k = lib().orc_solve_pixel(_p(W, _d), float(lam), _p(v, _d), _p(h, _d))
    return h, k


def is_tissue_u8(px, white_sum=660) -> bool:
    a = np.ascontiguousarray(np.asarray(px, dtype=np.uint8).reshape(3))
    return bool(lib().orc_is_tissue_u8(_p(a, _u8), int(white_sum)))


def is_tissue_f32(x0, x1, x2, white_sum=660) -> bool:
    return bool(lib().orc_is_tissue_f32(float(x0), float(x1), float(x2), int(white_sum)))


def densities_u8(img, W, i0=(255, 255, 255), lam=0.01, white_sum=660):
    """Returns (H (2, n) float64, mask (n,) uint8) for an (..., 3) uint8 image."""
    a = _img(img); n = a.shape[0]
    W = basis(W); i0 = _vec(i0, 3)
    H = np.empty((2, n)); m = np.empty(n, dtype=np.uint8)
    lib().orc_densities_u8(_p(a, _u8), n, _p(W, _d), _p(i0, _d), float(lam), int(white_sum), _p(H, _d), _p(m, _u8))
    return H, m


# ------------------------------------------------------------------ Eq. (3) percentile

def histogram(H, mask, hist_hi, bins=256):
    H = np.ascontiguousarray(H, dtype=np.float64); n = H.shape[1]
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    hh = _vec(hist_hi, 2); out = np.zeros((2, bins), dtype=np.uint64)
    lib().orc_histogram(_p(H, _d), None if m is None else _p(m, _u8), n, _p(hh, _d), int(bins), _p(out, _u64))
    return out


def percentile_hist(counts, hist_hi, q):
    c = np.ascontiguousarray(counts, dtype=np.uint64); P = C.c_double(); k = C.c_int()
    fl = lib().orc_percentile_hist(_p(c, _u64), c.size, float(hist_hi), float(q), C.byref(P), C.byref(k))
    return P.value, fl, k.value


def settle_range(H, mask, hist_hi, percentile=99.0, bins=256):
    """Ranges after the one automatic retry (a stain whose percentile lands in the last bin, at a
    range below 256, is counted again at twice its range).  Returns (ranges, retried-bits)."""
    H = np.ascontiguousarray(H, dtype=np.float64); n = H.shape[1]
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    hh = _vec(hist_hi, 2); out = np.zeros(2)
    bits = lib().orc_settle_range(_p(H, _d), None if m is None else _p(m, _u8), n, _p(hh, _d), int(bins),
                                  q_of(percentile), _p(out, _d))
    return [float(out[0]), float(out[1])], int(bits)


def percentile_exact(h, mask, q):
    h = np.ascontiguousarray(h, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    P = C.c_double(); idx = C.c_int64()
    fl = lib().orc_percentile_exact(_p(h, _d), None if m is None else _p(m, _u8), h.size, float(q),
                                    C.byref(P), C.byref(idx))
    return P.value, idx.value, fl


def q_of(percentile) -> float:
    """Percentile in (0, 100] as FP32 (as the library receives it) -> fraction in float64."""
    return float(np.float32(percentile)) / 100.0


# ------------------------------------------------------------------ Eqs. (3)-(4)

def normalize_u8(src, W_src, W_tgt, scale_tgt, i0_in=(255, 255, 255), i0_out=(255, 255, 255), lam=0.01,
                 white_sum=660, percentile=99.0, hist_hi=(4.0, 4.0), bins=256, auto_range=False):
    """Returns (out uint8 same shape, stats dict, hist (2, bins) uint64).  With auto_range the
    histogram is built over the ranges settle_range returns (stats "hist_hi", flags with
    RANGE_RETRY for a doubled stain)."""
    a = _img(src); n = a.shape[0]
    bits = 0
    if auto_range:
        H, m = densities_u8(src, W_src, i0_in, lam, white_sum)
        hist_hi, bits = settle_range(H, m, hist_hi, percentile, bins)
    out = np.empty_like(a); st = np.zeros(8); hist = np.zeros((2, bins), dtype=np.uint64)
    Ws, Wt = basis(W_src), basis(W_tgt)
    sc, ii, io, hh = _vec(scale_tgt, 2), _vec(i0_in, 3), _vec(i0_out, 3), _vec(hist_hi, 2)
    fl = lib().orc_normalize_u8(_p(a, _u8), n, _p(Ws, _d), _p(Wt, _d), _p(sc, _d), _p(ii, _d), _p(io, _d),
                                float(lam), int(white_sum), q_of(percentile), _p(hh, _d), int(bins),
                                _p(out, _u8), _p(st, _d), _p(hist, _u64))
    flags = st[4:6].astype(int) | np.array([RANGE_RETRY if bits >> j & 1 else 0 for j in range(2)])
    stats = {"P": st[0:2].copy(), "scale": st[2:4].copy(), "flags": flags, "n_tissue": int(st[6]),
             "status": fl, "hist_hi": list(hh)}
    return out.reshape(np.asarray(src).shape), stats, hist


def reconstruct_pixel(h, W_tgt, s, i0_out=(255, 255, 255)):
    h = _vec(h, 2); Wt = basis(W_tgt); s = _vec(s, 2); io = _vec(i0_out, 3); y = np.zeros(3)
    lib().orc_reconstruct_pixel(_p(h, _d), _p(Wt, _d), _p(s, _d), _p(io, _d), _p(y, _d))
    return y


def target_scale(tgt, W_tgt, i0=(255, 255, 255), lam=0.01, white_sum=660, percentile=99.0,
                 hist_hi=(4.0, 4.0), bins=256):
    """Eq. (3) numerator: the target's histogram percentile of each stain's density."""
    H, m = densities_u8(tgt, W_tgt, i0, lam, white_sum)
    hist = histogram(H, m, hist_hi, bins)
    q = q_of(percentile)
    P = [percentile_hist(hist[j], _vec(hist_hi, 2)[j], q)[0] for j in range(2)]
    return np.array(P), hist


# ------------------------------------------------------------------ basis estimation

def splitmix64(seed, t) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed & (2**64 - 1)), C.c_uint64(t)))


def recolor_u8(src, W_src, W_tgt, scale_tgt, P_src, i0_in=(255, 255, 255), i0_out=(255, 255, 255), lam=0.01,
               white_sum=660):
    """Eqs. 3-4 with given source percentiles.  Returns out uint8 of the source's shape."""
    a = _img(src); n = a.shape[0]
    out = np.empty_like(a)
    lib().orc_recolor_u8(_p(a, _u8), n, _p(basis(W_src), _d), _p(basis(W_tgt), _d), _p(_vec(scale_tgt, 2), _d),
                         _p(_vec(P_src, 2), _d), _p(_vec(i0_in, 3), _d), _p(_vec(i0_out, 3), _d), float(lam),
                         int(white_sum), _p(out, _u8))
    return out.reshape(np.asarray(src).shape)


def band_percentiles(img, W, band_rows, i0=(255, 255, 255), lam=0.01, white_sum=660, percentile=99.0,
                     hist_hi=(4.0, 4.0), bins=256):
    """Median of per-band percentiles.  Returns (median (2,), band_P (n_bands, 2), band_flags, flags)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    Hh, Ww = img.shape[0], img.shape[1]
    nb = (Hh + band_rows - 1) // band_rows
    bp = np.zeros((nb, 2)); bf = np.zeros((nb, 2), dtype=np.int32); med = np.zeros(2)
    f = lib().orc_band_percentiles(_p(img, _u8), Hh, Ww, _p(basis(W), _d), _p(_vec(i0, 3), _d), float(lam),
                                   int(white_sum), q_of(percentile), _p(_vec(hist_hi, 2), _d), int(bins),
                                   int(band_rows), _p(bp, _d), _p(bf, _i), _p(med, _d))
    return med, bp, bf, int(f)


def sample_percentile(img, W, n_s, seed, i0=(255, 255, 255), lam=0.01, white_sum=660, percentile=99.0,
                      max_cand=None):
    """Percentile of the sub-sampled non-white pixels' densities.  Returns (P (2,), kept, flags)."""
    a = _img(img); n = a.shape[0]
    max_cand = 64 * n_s if max_cand is None else max_cand
    P = np.zeros(2); kept = np.zeros(1, dtype=np.int64)
    f = lib().orc_sample_percentile(_p(a, _u8), n, _p(basis(W), _d), _p(_vec(i0, 3), _d), float(lam), int(white_sum),
                                    C.c_uint64(seed & (2**64 - 1)), int(n_s), int(max_cand), q_of(percentile),
                                    _p(P, _d), _p(kept, _i64))
    return P, int(kept[0]), int(f)


def exact_percentile(img, W, i0=(255, 255, 255), lam=0.01, white_sum=660, percentile=99.0):
    """Nearest-rank percentile of the densities of all non-white pixels.  Returns (P (2,), n, flags)."""
    a = _img(img); n = a.shape[0]
    P = np.zeros(2); nt = np.zeros(1, dtype=np.int64)
    f = lib().orc_exact_percentile_u8(_p(a, _u8), n, _p(basis(W), _d), _p(_vec(i0, 3), _d), float(lam),
                                      int(white_sum), q_of(percentile), _p(P, _d), _p(nt, _i64))
    return P, int(nt[0]), int(f)


def estimate_i0(img, n_s=100000, seed=0, white_sum=660, percentile=80.0, max_cand=None, default=(255.0, 255.0, 255.0)):
    """Channel-wise background intensity (Sec. 3.1 item 1).  Returns (i0 (3,) float64, kept)."""
    a = _img(img); n = a.shape[0]
    max_cand = 64 * n_s if max_cand is None else max_cand
    i0 = np.array(default, dtype=np.float64)
    k = lib().orc_estimate_i0(_p(a, _u8), n, int(white_sum), C.c_uint64(seed & (2**64 - 1)), int(n_s),
                              int(max_cand), q_of(percentile), _p(i0, _d))
    return i0, int(k)


def sample_tissue(img, n_s, seed, white_sum=660, max_cand=None):
    a = _img(img); n = a.shape[0]
    max_cand = 64 * n_s if max_cand is None else max_cand
    idx = np.zeros(max(n_s, 1), dtype=np.int64)
    k = lib().orc_sample_tissue(_p(a, _u8), n, int(white_sum), C.c_uint64(seed & (2**64 - 1)), int(n_s),
                                int(max_cand), _p(idx, _i64))
    return idx[:k]


def od_samples(img, idx, i0=(255, 255, 255)):
    """[3][n] FP64 optical densities of the sampled pixels (Eq. 1)."""
    a = _img(img)[idx]
    V = np.empty((3, len(idx)))
    for c in range(3):
        tab = np.array([od_u8(float(i0[c]), k) for k in range(256)])
        V[c] = tab[a[:, c]]
    return np.ascontiguousarray(V)


def nmf_objective(V, H, W, lam):
    V = np.ascontiguousarray(V, dtype=np.float64); H = np.ascontiguousarray(H, dtype=np.float64); Wb = basis(W)
    return lib().orc_nmf_objective(_p(V, _d), _p(H, _d), V.shape[1], _p(Wb, _d), float(lam))


def nmf(V, lam, T, W_init, percentile=99.0, trace=False):
    """Returns (W 6-vector fitted, sample_p99 (2,), objective trace or None)."""
    V = np.ascontiguousarray(V, dtype=np.float64); n = V.shape[1]
    W = basis(W_init).copy(); sp = np.zeros(2)
    tr = np.zeros(max(2 * T, 1)) if trace else None
    lib().orc_nmf(_p(V, _d), n, float(lam), int(T), _p(W, _d), None if tr is None else _p(tr, _d),
                  q_of(percentile), _p(sp, _d))
    return W, sp, tr


def stain_order_swap(W) -> bool:
    return bool(lib().orc_stain_order_swap(_p(basis(W), _d)))


def estimate_basis(img, n_s, seed, lam=0.1, T=50, W_init=None, i0=(255, 255, 255), white_sum=660,
                   percentile=99.0):
    """Sample -> OD -> sparse NMF -> stain order.  Returns (W 6-vector, sample_p99, idx)."""
    idx = sample_tissue(img, n_s, seed, white_sum)
    V = od_samples(img, idx, i0)
    if W_init is None:
        H0 = np.array([0.65, 0.70, 0.29]); E0 = np.array([0.07, 0.99, 0.11])
        W_init = np.stack([H0 / np.linalg.norm(H0), E0 / np.linalg.norm(E0)], axis=1)
        W_init = f32(W_init)
    W, sp, _ = nmf(V, lam, T, W_init, percentile)
    return W, sp, idx


# ------------------------------------------------------------------ differentiable float path

def forward_f32(x, W_src, W_tgt, scale_tgt, i0_in=(1, 1, 1), i0_out=(1, 1, 1), lam=0.01, white_sum=660,
                percentile=99.0):
    """x: (3, h, w) in [0, 1] (FP32 values widened to float64, or any float64 for finite differences).  Returns (y (3,h,w) float64, P (2,), istar (2,), H (2, n), flags)."""
    x = np.ascontiguousarray(x, dtype=np.float64); n = x.shape[1] * x.shape[2]
    y = np.empty((3, n)); P = np.zeros(2); ist = np.zeros(2, dtype=np.int64); H = np.empty((2, n))
    fl = lib().orc_forward_f32(_p(x, _d), n, _p(basis(W_src), _d), _p(basis(W_tgt), _d), _p(_vec(scale_tgt, 2), _d),
                               _p(_vec(i0_in, 3), _d), _p(_vec(i0_out, 3), _d), float(lam), int(white_sum),
                               q_of(percentile), _p(y, _d), _p(P, _d), _p(ist, _i64), _p(H, _d))
    return y.reshape(x.shape), P, ist, H, fl


def backward_f32(x, W_src, W_tgt, scale_tgt, grad_y, i0_in=(1, 1, 1), i0_out=(1, 1, 1), lam=0.01,
                 white_sum=660, percentile=99.0, istar=None):
    """Returns (grad_x (3,h,w) float64, grad_W_tgt 6-vector, grad_scale (2,), flags)."""
    x = np.ascontiguousarray(x, dtype=np.float64); n = x.shape[1] * x.shape[2]
    g = np.ascontiguousarray(grad_y, dtype=np.float64).reshape(3, n)
    gx = np.empty((3, n)); gW = np.zeros(6); gs = np.zeros(2)
    ist = None if istar is None else np.ascontiguousarray(istar, dtype=np.int64)
    fl = lib().orc_backward_f32(_p(x, _d), n, _p(basis(W_src), _d), _p(basis(W_tgt), _d), _p(_vec(scale_tgt, 2), _d),
                                _p(_vec(i0_in, 3), _d), _p(_vec(i0_out, 3), _d), float(lam), int(white_sum),
                                q_of(percentile), _p(g, _d), None if ist is None else _p(ist, _i64),
                                _p(gx, _d), _p(gW, _d), _p(gs, _d))
    return gx.reshape(x.shape), gW, gs, fl


def active_margin_f32(x, W_src, i0_in=(1, 1, 1), lam=0.01):
    """Per pixel (flat, n), the distance from an active-set change of Eq. (2): pixels with a tiny
    margin may be solved on another face in FP32 than in FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64); n = x.shape[1] * x.shape[2]
    m = np.empty(n)
    lib().orc_active_margin_f32(_p(x, _d), n, _p(basis(W_src), _d), _p(_vec(i0_in, 3), _d), float(lam), _p(m, _d))
    return m
