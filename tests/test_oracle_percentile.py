"""Pins of the oracle's Eq. (3) order statistic (histogram and exact modes) and of the full
normalisation of Eqs. (3)-(4): brute force, numpy's percentile, closed forms and invariants."""
import math

import numpy as np
import pytest

import synth


def test_histogram_brute_force(orc):
    rng = np.random.default_rng(11)
    n = 5000
    H = np.abs(rng.normal(0, 1.2, (2, n)))
    H[0, :50] = 0.0
    H[1, :7] = 10.0                       # beyond the top edge -> last bin
    mask = (rng.uniform(size=n) < 0.8).astype(np.uint8)
    hist = orc.histogram(H, mask, (4.0, 2.0), 256)
    for j, hi in enumerate((4.0, 2.0)):
        ref = np.zeros(256, dtype=np.uint64)
        for i in range(n):
            if mask[i]:
                k = min(255, int(math.floor(H[j, i] / (hi / 256))))
                ref[k] += 1
        assert np.array_equal(hist[j], ref)
    assert int(hist[0].sum()) == int(mask.sum())


def test_exact_percentile_matches_numpy(orc):
    rng = np.random.default_rng(12)
    for trial in range(40):
        n = int(rng.integers(1, 3000))
        h = rng.exponential(1.0, n)
        h[rng.uniform(size=n) < 0.2] = 0.0
        mask = (rng.uniform(size=n) < 0.7).astype(np.uint8)
        if mask.sum() == 0:
            continue
        q = [0.99, 0.5, 0.9, 1.0, 0.01][trial % 5]
        P, idx, fl = orc.percentile_exact(h, mask, q)
        ref = np.percentile(h[mask.astype(bool)], 100 * q, method="inverted_cdf")
        assert P == ref
        assert fl == orc.OK
        cand = np.nonzero(mask.astype(bool) & (h == P))[0]
        assert idx == cand[0]


def test_hist_percentile_within_one_bin_of_exact(orc):
    rng = np.random.default_rng(13)
    for trial in range(30):
        n = 20000
        H = np.abs(rng.normal(0.5, 0.6, (2, n)))
        mask = np.ones(n, np.uint8)
        hi = 4.0
        hist = orc.histogram(H, mask, (hi, hi), 256)
        for j in range(2):
            P, fl, k = orc.percentile_hist(hist[j], hi, 0.99)
            Pe, _, _ = orc.percentile_exact(H[j], mask, 0.99)
            assert abs(P - Pe) <= hi / 256 + 1e-15
            assert k == int(Pe // (hi / 256))


def test_hist_percentile_closed_form_uniform(orc):
    """Counts spread evenly inside each bin: the interpolated percentile is the exact quantile of
    the piecewise-uniform density, q * n / c_k positions into the crossing bin."""
    counts = np.zeros(256, dtype=np.uint64)
    counts[10] = 100
    counts[20] = 300
    counts[30] = 600
    # n = 1000, r = 990: crossing bin 30 after 400 below: 30 + 590/600 bins
    P, fl, k = orc.percentile_hist(counts, 4.0, 0.99)
    assert k == 30 and fl == orc.OK
    assert P == pytest.approx(4.0 / 256 * (30 + 590 / 600), rel=1e-15)
    # r exactly at a cumulative count: the crossing bin is the one that reaches it
    P, fl, k = orc.percentile_hist(counts, 4.0, 0.4)
    assert k == 20 and P == pytest.approx(4.0 / 256 * 21, rel=1e-15)


def test_hist_percentile_flags(orc):
    z = np.zeros(256, dtype=np.uint64)
    P, fl, _ = orc.percentile_hist(z, 4.0, 0.99)
    assert fl == orc.NO_TISSUE and P == 0.0
    c = z.copy(); c[0] = 1000
    _, fl, k = orc.percentile_hist(c, 4.0, 0.99)
    assert fl == orc.BIN0 and k == 0
    c = z.copy(); c[5] = 10; c[255] = 990
    _, fl, k = orc.percentile_hist(c, 4.0, 0.99)
    assert fl == orc.RANGE and k == 255


@pytest.mark.parametrize("hh", [(4.0, 2.0), (0.25, 8.0), (256.0, 0.5), (1.0, 1.0)])
def test_settle_range_counts_below_last_edge(orc, hh):
    """The range retry, pinned by counting: stain j's histogram percentile lies in the last bin
    exactly when fewer than q n tissue values lie below the last bin's lower edge 255 hh/256; then
    (and only below 256) its range doubles, once, and the other stain keeps its range."""
    rng = np.random.default_rng(17)
    q = float(np.float32(99.0)) / 100.0
    for trial in range(40):
        n = int(rng.integers(1, 400))
        scale = rng.choice([0.1, 1.0, 3.0, 30.0, 600.0], size=2)
        H = np.abs(rng.normal(0, 1, (2, n))) * scale[:, None]
        mask = (rng.uniform(size=n) < 0.9).astype(np.uint8)
        if mask.sum() == 0:
            mask[0] = 1
        ranges, bits = orc.settle_range(H, mask, hh)
        t = mask.astype(bool)
        for j in range(2):
            below = int((H[j, t] < 255.0 * hh[j] / 256.0).sum())
            overflow = below < q * int(t.sum())
            want = overflow and hh[j] < 256.0
            assert bool(bits >> j & 1) == want, (trial, j)
            assert ranges[j] == (2.0 * hh[j] if want else hh[j])
    # no tissue: nothing to retry
    ranges, bits = orc.settle_range(np.ones((2, 5)), np.zeros(5, dtype=np.uint8), hh)
    assert bits == 0 and ranges == list(hh)


def test_normalize_auto_range_equals_doubled_range(orc):
    """normalize with the retry equals normalize at the settled ranges, with RANGE_RETRY added."""
    d = synth.make_image(5, 60, 50)
    src = d["img"].numpy()
    W = d["W"]
    sc = np.array([0.9, 1.2])
    H, m = orc.densities_u8(src, orc.f32(orc.basis(W)))
    top = [float(np.quantile(H[j, m.astype(bool)], 0.995)) for j in range(2)]
    given = [2.0 ** math.floor(math.log2(top[0])), 4.0 * 2.0 ** math.ceil(math.log2(top[1]))]
    out_a, st_a, hist_a = orc.normalize_u8(src, orc.f32(orc.basis(W)), orc.f32(orc.basis(W)), sc, hist_hi=given,
                                           auto_range=True)
    assert st_a["hist_hi"] == [2.0 * given[0], given[1]]
    out_b, st_b, hist_b = orc.normalize_u8(src, orc.f32(orc.basis(W)), orc.f32(orc.basis(W)), sc,
                                           hist_hi=st_a["hist_hi"])
    assert np.array_equal(out_a, out_b) and np.array_equal(hist_a, hist_b)
    assert list(st_a["flags"]) == [st_b["flags"][0] | orc.RANGE_RETRY, st_b["flags"][1]]


# ------------------------------------------------------------------ Eqs. (3)-(4)

def noise_free_image(W, h, w, seed):
    """Pixels synthesised exactly in the cone of W (no background, no noise, no rounding loss
    beyond uint8): for lambda = 0 the densities are the solution of v = W h."""
    d = synth.make_image(seed, h, w, bg_frac=0.0, W=W, noise=0.0, keep_h=True)
    return d["img"].numpy()


def test_normalize_to_itself_is_identity(orc):
    """Reading of the identity property: lambda = 0, pixels synthesised in the cone of W without
    noise, W_tgt = W_src and scale_tgt = the source's own percentile -> every scale is exactly 1 and
    each pixel is rebuilt from its projection onto the cone.  The uint8 quantisation (<= 0.5 level
    per channel) is the only departure from the cone, so the output is within 1 level."""
    W = synth.reference_basis()
    img = noise_free_image(W, 40, 48, 21)
    P, _ = orc.target_scale(img, W, lam=0.0, white_sum=0)
    out, st, _ = orc.normalize_u8(img, W, W, P, lam=0.0, white_sum=0)
    assert np.array_equal(st["scale"], [1.0, 1.0])
    d = np.abs(out.astype(int) - img.astype(int))
    assert d.max() <= 1
    assert (d == 0).mean() > 0.9


def test_float_identity_exact_cone(orc):
    """Same property on the float path, where pixels can sit in the cone up to FP32 rounding:
    y = x to FP32 accuracy."""
    W = synth.reference_basis()
    rng = np.random.default_rng(25)
    h = rng.uniform(0, 2, (2, 20 * 20)) * (rng.uniform(size=(2, 400)) > 0.3)
    x = np.exp(-(W @ h)).reshape(3, 20, 20).astype(np.float32)
    y, P, ist, H, fl = orc.forward_f32(x, W, W, (1.0, 1.0), lam=0.0, white_sum=0)
    # scale_tgt = own percentile -> s = 1
    y, P2, _, _, _ = orc.forward_f32(x, W, W, P, lam=0.0, white_sum=0)
    assert np.array_equal(P, P2)
    assert np.abs(y - x).max() < 2e-6


def test_identity_through_projection(orc):
    """Any uint8 image, lambda = 0: output = rint(255 exp(-W h*)), the projection of each pixel's OD
    onto the cone of W, when W_tgt = W_src and scales are 1."""
    d = synth.make_image(22, 30, 30)
    img, W = d["img"].numpy(), d["W"]
    P, _ = orc.target_scale(img, W, lam=0.0)
    out, st, _ = orc.normalize_u8(img, W, W, P, lam=0.0)
    H, _ = orc.densities_u8(img, W, lam=0.0)
    ref = np.clip(np.rint(255 * np.exp(-(W @ H))), 0, 255).T.reshape(img.shape)
    assert np.array_equal(out, ref.astype(np.uint8))


def test_white_pixels_map_to_i0_out(orc):
    d = synth.make_image(23, 16, 16)
    img = d["img"].numpy().copy()
    img[:4] = 255
    Wt = synth.reference_basis()
    out, _, _ = orc.normalize_u8(img, d["W"], Wt, (1.0, 1.0), i0_out=(250, 240, 230))
    assert (out[:4] == np.array([250, 240, 230], np.uint8)).all()


def test_scale_equivariance(orc):
    """Multiplying scale_tgt by a multiplies every normalised OD v' by a (Eq. 3 is linear in it)."""
    d = synth.make_image(24, 24, 24)
    img, W = d["img"].numpy(), d["W"]
    Wt = synth.reference_basis()
    H, _ = orc.densities_u8(img, W)
    P, _ = orc.target_scale(img, W)
    for a in (0.5, 2.0):
        for i in range(0, H.shape[1], 17):
            s = np.array([1.3, 0.7])
            y1 = orc.reconstruct_pixel(H[:, i], Wt, s)
            y2 = orc.reconstruct_pixel(H[:, i], Wt, a * s)
            assert np.allclose(-np.log(y2 / 255), a * -np.log(y1 / 255), atol=1e-12)


def test_normalize_stats_consistent(orc):
    src, tgt = synth.config0(256)
    Ws, Wt = src["W"], tgt["W"]
    S, thist = orc.target_scale(tgt["img"].numpy(), Wt)
    out, st, hist = orc.normalize_u8(src["img"].numpy(), Ws, Wt, S)
    for j in range(2):
        P, fl, _ = orc.percentile_hist(hist[j], 4.0, orc.q_of(99.0))
        assert P == st["P"][j] and fl == st["flags"][j]
        assert st["scale"][j] == pytest.approx(S[j] / P, rel=1e-15)
    assert st["n_tissue"] == int(hist[0].sum())
    # the target's own scale equals its percentile: normalising the target with itself gives s = 1
    _, st2, _ = orc.normalize_u8(tgt["img"].numpy(), Wt, Wt, S)
    assert np.array_equal(st2["scale"], [1.0, 1.0])


def test_no_tissue_keeps_scale_one(orc):
    img = np.full((8, 8, 3), 250, np.uint8)
    W = synth.reference_basis()
    out, st, _ = orc.normalize_u8(img, W, W, (0.8, 0.9))
    assert st["status"] & orc.NO_TISSUE
    assert np.array_equal(st["scale"], [1.0, 1.0])
