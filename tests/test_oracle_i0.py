"""Pins of the oracle's channel-wise background intensity (Sec. 3.1 item 1): pixels with mean
intensity above 220 are sampled in the SplitMix64 draw order (itself pinned by the published
vectors in test_oracle_nmf_grad.py) and the 80th percentile of each channel is taken."""
import numpy as np
import pytest

import synth


def draws(orc, seed, n_px, count):
    return [(orc.splitmix64(seed, t) * n_px) >> 64 for t in range(count)]


def test_matches_numpy_nearest_rank(orc):
    """Brute force: the first n_s background draws, then numpy's inverted-CDF percentile (the
    nearest-rank definition: the k-th smallest value, k = ceil(q n))."""
    d = synth.make_image(5, 96, 80, bg_frac=0.5)
    img = d["img"].numpy()
    flat = img.reshape(-1, 3).astype(int)
    n_s = 700
    i0, kept = orc.estimate_i0(img, n_s, seed=123)
    assert kept == n_s
    cand = draws(orc, 123, flat.shape[0], 64 * n_s)
    bg = [c for c in cand if flat[c].sum() > 660][:n_s]
    ref = np.percentile(flat[bg], 80, axis=0, method="inverted_cdf")
    assert np.array_equal(i0, ref)
    # other percentiles
    for q in (1.0, 50.0, 99.0, 100.0):
        i0q, _ = orc.estimate_i0(img, n_s, seed=123, percentile=q)
        assert np.array_equal(i0q, np.percentile(flat[bg], q, axis=0, method="inverted_cdf")), q


def test_constant_background_and_extremes(orc):
    img = np.zeros((40, 50, 3), np.uint8)
    img[...] = (240, 245, 250)
    i0, kept = orc.estimate_i0(img, 100, seed=9)
    assert kept == 100 and list(i0) == [240, 245, 250]
    # percentile 100 is the largest sampled value, a tiny percentile the smallest
    rng = np.random.default_rng(3)
    img = rng.integers(225, 256, size=(64, 64, 3), dtype=np.uint8)
    flat = img.reshape(-1, 3).astype(int)
    cand = draws(orc, 4, flat.shape[0], 64 * 300)
    bg = np.array([c for c in cand if flat[c].sum() > 660][:300])
    hi, _ = orc.estimate_i0(img, 300, seed=4, percentile=100.0)
    lo, _ = orc.estimate_i0(img, 300, seed=4, percentile=0.001)
    assert np.array_equal(hi, flat[bg].max(0)) and np.array_equal(lo, flat[bg].min(0))


def test_threshold_is_strict_and_excludes_ties(orc):
    """Mean exactly 220 (sum 660) is neither tissue nor background; nothing found leaves i0 as is."""
    img = np.zeros((16, 16, 3), np.uint8)
    img[...] = (220, 220, 220)
    i0, kept = orc.estimate_i0(img, 50, seed=1)
    assert kept == 0 and list(i0) == [255, 255, 255]
    img[...] = (221, 220, 220)
    i0, kept = orc.estimate_i0(img, 50, seed=1)
    assert kept == 50 and list(i0) == [221, 220, 220]
    # a tissue-only image: nothing kept, the caller's default survives
    img[...] = (100, 80, 120)
    i0, kept = orc.estimate_i0(img, 50, seed=1, default=(250.0, 251.0, 252.0))
    assert kept == 0 and list(i0) == [250, 251, 252]


def test_short_sample_and_budget(orc):
    """Fewer background pixels than requested within 64 n_s draws: all found ones are used."""
    img = np.full((32, 32, 3), 90, np.uint8)
    img[0, :4] = (230, 240, 250)
    flat = img.reshape(-1, 3).astype(int)
    i0, kept = orc.estimate_i0(img, 1000, seed=11)
    cand = draws(orc, 11, flat.shape[0], 64 * 1000)
    assert kept == sum(1 for c in cand if flat[c].sum() > 660)
    assert list(i0) == [230, 240, 250]
    i0b, keptb = orc.estimate_i0(img, 1000, seed=11, max_cand=100)
    assert keptb == sum(1 for c in cand[:100] if flat[c].sum() > 660)
