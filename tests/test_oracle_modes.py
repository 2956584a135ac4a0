"""Pins of the oracle's paper-compatible percentile modes: the median of per-patch (row band)
percentiles (Sec. 3.2 items 3-4), the percentile of the sub-sampled non-white pixels (Sec. 3.1
item 2), and recolouring from given percentiles (Eqs. 3-4)."""
import numpy as np
import pytest

import synth


def global_P(orc, img, W, lam=0.01):
    _, st, _ = orc.normalize_u8(img, W, W, np.ones(2), lam=lam)
    return st["P"]


def test_single_band_equals_global(orc):
    d = synth.make_image(2, 150, 220)
    img = d["img"].numpy()
    W = orc.f32(orc.basis(d["W"]))
    med, bp, bf, f = orc.band_percentiles(img, W, 150)
    assert bp.shape == (1, 2) and f == 0
    assert np.array_equal(med, global_P(orc, img, W))
    med2, _, _, _ = orc.band_percentiles(img, W, 1000)
    assert np.array_equal(med2, med)


def test_band_median_closed_form(orc):
    """Bands of one tissue colour each: every density of a band lies in one bin k, so the band's
    percentile is width * (k + q); white bands hold no tissue and are skipped; the median is numpy's
    (middle value, or the mean of the two middle values)."""
    colours = [(120, 60, 140), (200, 120, 190), (90, 40, 110), (250, 250, 250), (160, 100, 170), (60, 30, 90)]
    W = orc.f32(orc.basis(synth.reference_basis()))
    for n_bands in (5, 6):   # odd / even count of tissue bands (the white band excluded)
        cols = [c for c in colours[:n_bands + 1]]
        img = np.concatenate([np.broadcast_to(np.array(c, np.uint8), (7, 9, 3)) for c in cols]).copy()
        med, bp, bf, f = orc.band_percentiles(img, W, 7)
        width = 4.0 / 256
        expect = []
        for b, c in enumerate(cols):
            if sum(c) >= 660:
                assert (bf[b] & 1).all()   # no tissue
                continue
            H, _ = orc.densities_u8(np.array([[c]], np.uint8), W)
            k = np.minimum(np.floor(H[:, 0] / width), 255)
            assert np.allclose(bp[b], width * (k + 0.99), rtol=0, atol=1e-12)
            expect.append(bp[b])
        assert np.array_equal(med, np.median(np.array(expect), axis=0))


def test_no_tissue_band_median(orc):
    img = np.full((20, 10, 3), 245, np.uint8)
    med, bp, bf, f = orc.band_percentiles(img, orc.f32(orc.basis(synth.reference_basis())), 4)
    assert f & 1 and list(med) == [0.0, 0.0] and (bf & 1).all()


def test_sample_percentile_brute_force(orc):
    d = synth.make_image(8, 120, 130)
    img = d["img"].numpy()
    W = orc.f32(orc.basis(d["W"]))
    flat = img.reshape(-1, 3)
    n_s = 3000
    P, kept, f = orc.sample_percentile(img, W, n_s, seed=21)
    assert kept == n_s and f == 0
    cand = [(orc.splitmix64(21, t) * flat.shape[0]) >> 64 for t in range(64 * n_s)]
    idx = [c for c in cand if int(flat[c].astype(int).sum()) < 660][:n_s]
    H, _ = orc.densities_u8(flat[idx].reshape(-1, 1, 3), W)
    for j in range(2):
        assert P[j] == np.percentile(H[j], 99, method="inverted_cdf")
    # a constant tissue colour: the percentile is that colour's density, whatever q
    img2 = np.broadcast_to(np.array((130, 70, 150), np.uint8), (30, 30, 3)).copy()
    H2, _ = orc.densities_u8(img2[:1, :1], W)
    for q in (1.0, 50.0, 99.0):
        P2, _, _ = orc.sample_percentile(img2, W, 100, seed=1, percentile=q)
        assert np.array_equal(P2, H2[:, 0])
    P3, kept3, f3 = orc.sample_percentile(np.full((8, 8, 3), 250, np.uint8), W, 10, seed=1)
    assert kept3 == 0 and f3 & 1 and list(P3) == [0.0, 0.0]


def test_recolor_given_percentiles(orc):
    """With the global histogram percentile given, recolouring equals the two-pass normalisation;
    multiplying P and the target scale by 2 changes nothing (s = scale / P exactly)."""
    src = synth.make_image(0, 90, 110)
    tgt = synth.make_image(1, 40, 40)
    Ws, Wt = orc.f32(orc.basis(src["W"])), orc.f32(orc.basis(tgt["W"]))
    sc = np.array([1.7, 0.9])
    img = src["img"].numpy()
    out, st, _ = orc.normalize_u8(img, Ws, Wt, sc)
    rec = orc.recolor_u8(img, Ws, Wt, sc, st["P"])
    assert np.array_equal(rec, out)
    rec2 = orc.recolor_u8(img, Ws, Wt, 2 * sc, 2 * np.asarray(st["P"]))
    assert np.array_equal(rec2, out)
    # P not > 0 keeps the stain unscaled (scale 1)
    one = orc.recolor_u8(img, Ws, Wt, sc, [0.0, 0.0])
    ref = orc.recolor_u8(img, Ws, Wt, [1.0, 1.0], [1.0, 1.0])
    assert np.array_equal(one, ref)


def test_exact_percentile_pins(orc):
    """The exact order statistic over all non-white pixels: numpy's inverted-CDF percentile of the
    tissue densities; within one bin width of the histogram percentile (Eq. 3 read through the
    histogram); white pixels do not enter; q = 100 gives the maximum, a tiny q the minimum; a
    constant colour gives its own density for any q; no tissue gives 0 and the flag."""
    d = synth.make_image(5, 97, 131)
    img = d["img"].numpy()
    W = orc.f32(orc.basis(d["W"]))
    P, n, f = orc.exact_percentile(img, W)
    H, m = orc.densities_u8(img, W)
    t = m.astype(bool)
    assert n == int(t.sum()) and f == 0
    for j in range(2):
        assert P[j] == np.percentile(H[j][t], 99, method="inverted_cdf")
        # nearest rank by a plain sort of the tissue densities
        vals = sorted(H[j][t].tolist())
        k = max(1, int(np.ceil(orc.q_of(99.0) * n)))
        assert P[j] == vals[k - 1]
    Ph = global_P(orc, img, W)
    assert np.all(np.abs(P - Ph) <= 4.0 / 256)
    Pmax, _, _ = orc.exact_percentile(img, W, percentile=100.0)
    Pmin, _, _ = orc.exact_percentile(img, W, percentile=1e-6)
    assert np.array_equal(Pmax, H[:, t].max(1)) and np.array_equal(Pmin, H[:, t].min(1))
    # extra white rows change nothing
    img_w = np.concatenate([img, np.full((13, 131, 3), 250, np.uint8)])
    assert np.array_equal(orc.exact_percentile(img_w, W)[0], P)
    # white_sum = 0: every pixel counts
    P0, n0, _ = orc.exact_percentile(img, W, white_sum=0)
    assert n0 == img.shape[0] * img.shape[1]
    assert P0[0] == np.percentile(H[0], 99, method="inverted_cdf")
    col = np.broadcast_to(np.array((140, 80, 160), np.uint8), (9, 11, 3)).copy()
    Hc, _ = orc.densities_u8(col[:1, :1], W)
    for q in (0.5, 50.0, 100.0):
        assert np.array_equal(orc.exact_percentile(col, W, percentile=q)[0], Hc[:, 0])
    Pw, nw, fw = orc.exact_percentile(np.full((5, 5, 3), 252, np.uint8), W)
    assert nw == 0 and fw & 1 and list(Pw) == [0.0, 0.0]
