"""Pins of the oracle's basis estimation (sampling, sparse NMF of Eq. 2, stain order) and of its
hand-derived adjoint of the differentiable float path (finite differences of its own forward)."""
import math

import numpy as np
import pytest

import synth


def angle_deg(a, b):
    a = np.asarray(a) / np.linalg.norm(a); b = np.asarray(b) / np.linalg.norm(b)
    return math.degrees(math.acos(min(1.0, float(a @ b))))


# ------------------------------------------------------------------ sampling

def test_splitmix64_published_vectors(orc):
    """First outputs of the SplitMix64 reference generator started from state 0 (Steele, Lea &
    Flood 2014; the widely used reference C implementation), stored in tests/golden."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.json")))
    for t, h in enumerate(g["outputs_hex"]):
        assert orc.splitmix64(g["seed"], t) == int(h, 16)


def test_sampler_properties(orc):
    d = synth.make_image(31, 64, 80)
    img = d["img"].numpy()
    flat = img.reshape(-1, 3).astype(int)
    idx = orc.sample_tissue(img, 500, seed=77)
    assert len(idx) == 500
    assert (idx >= 0).all() and (idx < flat.shape[0]).all()
    assert (flat[idx].sum(1) < 660).all()
    # deterministic, and the first accepted candidates in draw order
    assert np.array_equal(idx, orc.sample_tissue(img, 500, seed=77))
    cand = [(orc.splitmix64(77, t) * flat.shape[0]) >> 64 for t in range(3000)]
    acc = [c for c in cand if flat[c].sum() < 660][:500]
    assert np.array_equal(idx, acc)
    # an all-white image yields nothing within the candidate budget
    assert len(orc.sample_tissue(np.full((8, 8, 3), 250, np.uint8), 10, seed=1)) == 0


def test_sampler_uniform(orc):
    img = np.zeros((100, 100, 3), np.uint8)
    idx = orc.sample_tissue(img, 40000, seed=5)
    counts = np.bincount(idx // 1000, minlength=10)
    assert counts.min() > 3700 and counts.max() < 4300


# ------------------------------------------------------------------ sparse NMF

def synth_od(W, n, seed, minor=0.15, noise=0.0, pure=False):
    rng = np.random.default_rng(seed)
    dom = rng.integers(0, 2, n)
    hd = rng.uniform(0.1, 2.0, n)
    hm = 0.0 if pure else rng.uniform(0, minor, n) * hd
    H = np.zeros((2, n))
    H[dom, np.arange(n)] = hd
    H[1 - dom, np.arange(n)] = hm
    V = W @ H + rng.normal(0, noise, (3, n))
    return np.clip(V, 0, None)


def test_nmf_objective_pins(orc):
    """The Eq. (2) objective ||V - W H||_F^2 + lambda sum(H) that the monotonicity pin below rests
    on, against values the definition fixes: a hand-computed integer case, H = 0, an exact
    factorisation V = W H (only the penalty remains), the slope in lambda, and a numpy evaluation
    of the same definition on random data."""
    # V columns (1,2,3) and (0,1,2); W = unit R and G axes; H columns (1,1) and (0,1):
    # residuals (0,1,3) and (0,0,2) -> 1 + 9 + 4 = 14, plus lambda * 3
    V = np.array([[1.0, 0.0], [2.0, 1.0], [3.0, 2.0]])
    W = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    H = np.array([[1.0, 0.0], [1.0, 1.0]])
    assert orc.nmf_objective(V, H, W, 0.5) == 15.5
    assert orc.nmf_objective(V, H, W, 0.0) == 14.0
    rng = np.random.default_rng(60)
    Wr = synth.jitter_basis(rng, 5)
    Hr = rng.uniform(0, 2, (2, 500))
    Vr = rng.uniform(0, 3, (3, 500))
    assert np.isclose(orc.nmf_objective(Vr, np.zeros((2, 500)), Wr, 0.3), (Vr ** 2).sum(), rtol=1e-13)
    Vx = Wr @ Hr
    assert np.isclose(orc.nmf_objective(Vx, Hr, Wr, 0.1), 0.1 * Hr.sum(), rtol=1e-12)
    f1, f2 = orc.nmf_objective(Vr, Hr, Wr, 0.1), orc.nmf_objective(Vr, Hr, Wr, 0.7)
    assert np.isclose(f2 - f1, 0.6 * Hr.sum(), rtol=1e-10)
    assert np.isclose(f1, ((Vr - Wr @ Hr) ** 2).sum() + 0.1 * Hr.sum(), rtol=1e-13)


def test_nmf_objective_monotone(orc):
    W = synth.jitter_basis(np.random.default_rng(40), 5)
    V = synth_od(W, 4000, 41, noise=0.03)
    W0 = synth.jitter_basis(np.random.default_rng(42), 15)
    Wf, sp, tr = orc.nmf(V, 0.1, 30, W0, trace=True)
    d = np.diff(tr)
    assert d.max() <= 1e-9 * tr[0]
    assert tr[-1] < tr[0]


def test_nmf_separable_recovery(orc):
    """Pure-stain pixels: both stain directions are in the data, and the fitted unit columns are
    exactly those directions."""
    W = synth.jitter_basis(np.random.default_rng(43), 5)
    V = synth_od(W, 3000, 44, pure=True)
    Wf, _, _ = orc.nmf(V, 0.1, 200, synth.reference_basis())
    Wf = Wf.reshape(2, 3).T
    for j in range(2):
        assert angle_deg(Wf[:, j], W[:, j]) < 0.05


def test_nmf_generator_recovery(orc):
    """Generator-like mixtures (minor stain <= 15% of the dominant one): within 3 degrees."""
    for seed in (45, 46, 47):
        W = synth.jitter_basis(np.random.default_rng(seed), 5)
        V = synth_od(W, 20000, seed + 100, noise=0.02)
        Wf, sp, _ = orc.nmf(V, 0.1, 50, synth.reference_basis())
        Wf = Wf.reshape(2, 3).T
        assert np.allclose(np.linalg.norm(Wf, axis=0), 1.0, atol=1e-12)
        assert (Wf >= 0).all()
        for j in range(2):
            assert angle_deg(Wf[:, j], W[:, j]) < 3.0
        H = np.array([orc.solve_pixel(Wf, 0.1, V[:, i])[0] for i in range(V.shape[1])]).T
        for j in range(2):
            assert sp[j] == np.percentile(H[j], 99.0, method="inverted_cdf")


def test_stain_order_red_minus_blue(orc):
    """Hematoxylin (larger OD in red than blue) comes first, whatever the initial order."""
    W = synth.jitter_basis(np.random.default_rng(48), 5)
    V = synth_od(W, 5000, 49, noise=0.01)
    Wf, _, _ = orc.nmf(V, 0.1, 60, synth.reference_basis()[:, ::-1])
    Wf = Wf.reshape(2, 3).T
    assert Wf[0, 0] - Wf[2, 0] > Wf[0, 1] - Wf[2, 1]
    assert angle_deg(Wf[:, 0], W[:, 0]) < 3.0
    assert orc.stain_order_swap(synth.reference_basis()[:, ::-1])
    assert not orc.stain_order_swap(synth.reference_basis())


def test_estimate_basis_on_image(orc):
    src, _ = synth.config0(256)
    W, sp, idx = orc.estimate_basis(src["img"].numpy(), 4000, seed=9, lam=0.1, T=50)
    Wm = W.reshape(2, 3).T
    for j in range(2):
        assert angle_deg(Wm[:, j], src["W"][:, j]) < 4.0
    assert (sp > 0).all()


# ------------------------------------------------------------------ adjoint of the float path

def _fwd(orc, x, Ws, Wt, S, lam, white_sum=660):
    return orc.forward_f32(x, Ws, Wt, S, lam=lam, white_sum=white_sum)


def _dloss(wts, yp, ym):
    """L(+) - L(-) for L = sum(w * y^2), summed from per-element differences (exact where an
    element does not change), so that the difference quotient is not lost in the rounding of two
    large sums."""
    return float((wts * (yp - ym) * (yp + ym)).sum())


def _crop32(seed):
    """A 32 x 32 crop of the float workload's generator (the benchmark's 512 x 512 images are made
    of the same field), as FP32 values in [0, 1] widened to float64."""
    d = synth.make_image(seed, 96, 96)
    x = d["img"][40:72, 24:56].numpy().transpose(2, 0, 1).astype(np.float32) / np.float32(255.0)
    return np.ascontiguousarray(x.astype(np.float64)), d["W"]


@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_backward_matches_finite_differences(orc, lam):
    """FP64 central differences of the oracle's own forward, eps = 1e-6, on a 32 x 32 crop, at
    pixels away from active-set switches and rank swaps; L = sum(w * y^2), so dL/dy = 2 w y."""
    x, Ws = _crop32(50)
    Wt = synth.target_bases(1, 51, 10.0)[0]
    S = np.array([0.9, 1.1])
    wts = np.random.default_rng(52).uniform(0, 1, x.shape)
    y, P, ist, H, fl = _fwd(orc, x, Ws, Wt, S, lam)
    gx, gW, gs, fl = orc.backward_f32(x, Ws, Wt, S, 2.0 * wts * y, lam=lam)
    eps = 1e-6
    n = x.shape[1] * x.shape[2]
    margin = orc.active_margin_f32(x, Ws, lam=lam)
    checked = 0
    for i in list(range(0, n, 5)) + list(ist):
        if margin[i] < 1e-4:
            continue           # an active-set switch within reach of the perturbation
        for c in range(3):
            xc = x.reshape(3, -1)[c, i]
            if xc >= 1.0 - 1e-4 or xc <= 1.0 / 255 + 1e-4:
                continue       # the OD clamp's kinks (x = 1 and x = 1/255): one-sided derivatives
            xp = x.copy(); xm = x.copy()
            xp.reshape(3, -1)[c, i] += eps; xm.reshape(3, -1)[c, i] -= eps
            rp, rm = _fwd(orc, xp, Ws, Wt, S, lam), _fwd(orc, xm, Ws, Wt, S, lam)
            if not (np.array_equal(rp[2], ist) and np.array_equal(rm[2], ist)):
                continue       # the selected order statistic changed pixel: not differentiable here
            fd = _dloss(wts, rp[0], rm[0]) / (2 * eps)
            an = gx.reshape(3, -1)[c, i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, c, fd, an)
            checked += 1
    assert checked > 300
    # the selected pixels themselves carry the order-statistic term
    for j in range(2):
        k = int(ist[j])
        if margin[k] >= 1e-4:
            for c in range(3):
                xp = x.copy(); xm = x.copy()
                xp.reshape(3, -1)[c, k] += eps; xm.reshape(3, -1)[c, k] -= eps
                rp, rm = _fwd(orc, xp, Ws, Wt, S, lam), _fwd(orc, xm, Ws, Wt, S, lam)
                if np.array_equal(rp[2], ist) and np.array_equal(rm[2], ist):
                    fd = _dloss(wts, rp[0], rm[0]) / (2 * eps)
                    assert abs(fd - gx.reshape(3, -1)[c, k]) <= 1e-6 * max(1.0, abs(fd)), (j, c)
    Wb = orc.basis(Wt)
    for k in range(6):
        Wp = Wb.copy(); Wm = Wb.copy(); Wp[k] += eps; Wm[k] -= eps
        fd = _dloss(wts, _fwd(orc, x, Ws, Wp, S, lam)[0], _fwd(orc, x, Ws, Wm, S, lam)[0]) / (2 * eps)
        assert abs(fd - gW[k]) <= 1e-6 * max(1.0, abs(gW[k])), (k, fd, gW[k])
    for j in range(2):
        Sp = S.copy(); Sm = S.copy(); Sp[j] += eps; Sm[j] -= eps
        fd = _dloss(wts, _fwd(orc, x, Ws, Wt, Sp, lam)[0], _fwd(orc, x, Ws, Wt, Sm, lam)[0]) / (2 * eps)
        assert abs(fd - gs[j]) <= 1e-6 * max(1.0, abs(gs[j])), (j, fd, gs[j])


def test_backward_selected_pixel_carries_percentile_term(orc):
    """The pixel holding the order statistic gets the extra term -(s/P) dL/ds through its density;
    zeroing every other pixel's weight leaves it the only non-zero input gradient besides itself."""
    d = synth.make_image(53, 12, 12)
    x = np.ascontiguousarray(d["img"].numpy().transpose(2, 0, 1).astype(np.float64) / 255.0)
    Ws = d["W"]; Wt = synth.reference_basis(); S = np.array([1.0, 1.0])
    y, P, ist, H, fl = orc.forward_f32(x, Ws, Wt, S)
    k = int(ist[0])
    other = (k + 5) % H.shape[1]
    gy = np.zeros(x.shape)
    gy.reshape(3, -1)[:, other] = 1.0
    gx, gW, gs, _ = orc.backward_f32(x, Ws, Wt, S, gy)
    nz = np.nonzero(np.abs(gx.reshape(3, -1)).sum(0))[0]
    assert set(nz.tolist()) <= {k, other, int(ist[1])}
    if H[0, other] > 0 and H[0, k] > 0:
        assert k in nz.tolist()
