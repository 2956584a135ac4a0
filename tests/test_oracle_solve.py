"""Pins of the oracle's Eq. (1) optical density and Eq. (2) per-pixel density solve.

Every check here compares the oracle with something other than its own formula: optimality
(KKT) conditions, brute-force search, SciPy / scikit-learn solvers, closed forms for special bases,
and symmetries the problem must have.
"""
import math

import numpy as np
import pytest
from scipy.optimize import nnls

import synth


def rand_basis(rng, deg=5.0):
    return synth.jitter_basis(rng, deg)


def objective(W, lam, v, h):
    r = v - W @ h
    return float(r @ r + lam * h.sum())


# ------------------------------------------------------------------ Eq. (1)

def test_od_closed_forms(orc):
    assert orc.od_u8(255, 255) == 0.0
    assert orc.od_u8(255, 85) == pytest.approx(math.log(3.0), abs=1e-15)
    assert orc.od_u8(255, 1) == pytest.approx(math.log(255.0), abs=1e-15)
    assert orc.od_u8(255, 0) == orc.od_u8(255, 1)          # intensity 0 read as 1
    assert orc.od_u8(200, 250) == 0.0                      # above i0: clamped at zero
    assert orc.od_u8(240, 120) == pytest.approx(math.log(2.0), abs=1e-15)
    assert orc.od_f(1.0, 1.0) == 0.0
    assert orc.od_f(1.0, 0.5) == pytest.approx(math.log(2.0), abs=1e-15)
    assert orc.od_f(1.0, 0.0) == pytest.approx(math.log(255.0), abs=1e-14)


def test_od_monotone(orc):
    vals = [orc.od_u8(255, k) for k in range(1, 256)]
    assert all(a > b for a, b in zip(vals, vals[1:]))


# ------------------------------------------------------------------ Eq. (2), W fixed

def test_kkt_conditions_random(orc):
    """Stationarity / complementary slackness of min ||v - W h||^2 + lam 1^T h over h >= 0."""
    rng = np.random.default_rng(1)
    for trial in range(3000):
        W = rand_basis(rng)
        lam = [0.0, 0.01, 0.1, 0.5][trial % 4]
        v = rng.uniform(0, 3, 3) if trial % 3 else W @ rng.uniform(-0.5, 2.5, 2) + rng.normal(0, 0.05, 3)
        h, _ = orc.solve_pixel(W, lam, v)
        grad = 2 * W.T @ (W @ h - v) + lam
        assert (h >= 0).all()
        for j in range(2):
            if h[j] > 0:
                assert abs(grad[j]) < 1e-9, (trial, h, grad)
            else:
                assert grad[j] > -1e-9, (trial, h, grad)


def test_brute_force_grid(orc):
    """Exhaustive grid over [0, 4]^2 never beats the oracle's minimiser."""
    rng = np.random.default_rng(2)
    g = np.arange(0, 4.0001, 1e-2)
    A, B = np.meshgrid(g, g, indexing="ij")
    for trial in range(60):
        W = rand_basis(rng)
        lam = [0.0, 0.01, 0.1][trial % 3]
        v = np.clip(W @ rng.uniform(-0.3, 2.0, 2) + rng.normal(0, 0.1, 3), 0, None)
        h, _ = orc.solve_pixel(W, lam, v)
        R = v[:, None, None] - (W[:, 0, None, None] * A + W[:, 1, None, None] * B)
        F = (R ** 2).sum(0) + lam * (A + B)
        fbest = objective(W, lam, v, h)
        assert fbest <= F.min() + 1e-12
        i, j = np.unravel_index(F.argmin(), F.shape)
        # strictly convex: the grid argmin lies within a few grid steps of the true minimiser
        assert abs(g[i] - h[0]) < 0.1 and abs(g[j] - h[1]) < 0.1


def test_lambda0_exact_recovery(orc):
    """lambda = 0 and v = W h with h >= 0: h is recovered exactly (the pseudo-inverse case)."""
    rng = np.random.default_rng(3)
    for _ in range(2000):
        W = rand_basis(rng)
        h0 = rng.uniform(0, 3, 2) * (rng.uniform(0, 1, 2) > 0.2)
        h, _ = orc.solve_pixel(W, 0.0, W @ h0)
        assert np.allclose(h, h0, atol=1e-12)
        if (h0 > 0).all():
            assert np.allclose(h, np.linalg.pinv(W) @ (W @ h0), atol=1e-12)


def test_orthogonal_basis_soft_threshold(orc):
    """G = I: the problem separates into scalar lasso problems, h_j = max(0, w_j^T v - lam/2)."""
    rng = np.random.default_rng(4)
    W = np.array([[1.0, 0.0], [0.0, 0.6], [0.0, 0.8]])
    for _ in range(500):
        lam = rng.uniform(0, 0.5)
        v = rng.uniform(0, 2, 3)
        h, _ = orc.solve_pixel(W, lam, v)
        assert np.allclose(h, np.maximum(0.0, W.T @ v - lam / 2), atol=1e-13)


def test_scipy_nnls_lambda0(orc):
    rng = np.random.default_rng(5)
    for _ in range(500):
        W = rand_basis(rng)
        v = rng.uniform(0, 3, 3)
        h, _ = orc.solve_pixel(W, 0.0, v)
        ref, _ = nnls(W, v)
        assert np.allclose(h, ref, atol=1e-10)


def test_sklearn_positive_lasso(orc):
    """sklearn's Lasso minimises ||y - X w||^2 / (2 n) + alpha |w|_1 with n = 3 rows, so
    alpha = lam / 6 reproduces Eq. (2)'s per-pixel objective."""
    from sklearn.linear_model import Lasso
    rng = np.random.default_rng(6)
    for _ in range(150):
        W = rand_basis(rng)
        lam = rng.choice([0.01, 0.1, 0.3])
        v = np.clip(W @ rng.uniform(0, 2.0, 2) + rng.normal(0, 0.1, 3), 0, None)
        h, _ = orc.solve_pixel(W, lam, v)
        m = Lasso(alpha=lam / 6.0, positive=True, fit_intercept=False, tol=1e-14, max_iter=100000)
        m.fit(W, v)
        assert np.allclose(h, m.coef_, atol=1e-8)


def test_white_pixel_zero_density(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        W = rand_basis(rng)
        for lam in (0.0, 0.01, 0.1):
            h, _ = orc.solve_pixel(W, lam, np.zeros(3))
            assert (h == 0).all()
    W = synth.reference_basis()
    H, m = orc.densities_u8(np.full((4, 3), 255, np.uint8), W)
    assert (H == 0).all() and (m == 0).all()


def test_column_swap_symmetry(orc):
    rng = np.random.default_rng(8)
    for _ in range(500):
        W = rand_basis(rng)
        v = rng.uniform(0, 3, 3)
        h, _ = orc.solve_pixel(W, 0.05, v)
        hs, _ = orc.solve_pixel(W[:, ::-1], 0.05, v)
        assert np.allclose(h, hs[::-1], atol=1e-12)


def test_positive_homogeneity(orc):
    """h(t v, t lam) = t h(v, lam) for t > 0 (the objective scales by t^2)."""
    rng = np.random.default_rng(9)
    for _ in range(300):
        W = rand_basis(rng)
        v = rng.uniform(0, 2, 3)
        t = rng.uniform(0.2, 5)
        h, _ = orc.solve_pixel(W, 0.1, v)
        ht, _ = orc.solve_pixel(W, 0.1 * t, t * v)
        assert np.allclose(ht, t * h, atol=1e-11)


def test_densities_image_matches_pixelwise(orc):
    d = synth.make_image(3, 24, 20)
    img = d["img"].numpy()
    W = d["W"]
    H, m = orc.densities_u8(img, W, lam=0.01)
    flat = img.reshape(-1, 3)
    for i in range(0, flat.shape[0], 37):
        v = [orc.od_u8(255, int(c)) for c in flat[i]]
        h, _ = orc.solve_pixel(W, 0.01, v)
        assert np.array_equal(h, H[:, i])
        assert m[i] == (int(flat[i].astype(int).sum()) < 660)


def test_tissue_mask_thresholds(orc):
    assert orc.is_tissue_u8([219, 220, 220])          # 659
    assert not orc.is_tissue_u8([220, 220, 220])      # 660: white
    assert orc.is_tissue_u8([255, 255, 255], white_sum=0)
    assert orc.is_tissue_f32(219 / 255, 220 / 255, 220 / 255)
    assert not orc.is_tissue_f32(1.0, 1.0, 1.0)
