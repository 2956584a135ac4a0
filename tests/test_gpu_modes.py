"""GPU parity of the paper-compatible percentile modes with the FP64 oracle: the median of per-band
percentiles (exact band histograms, so the same FP64 percentile formula gives identical values),
the percentile of the sub-sampled non-white pixels (same draws; FP64 densities on both sides, so
the selected value agrees to the last bits), and recolouring from given percentiles (uint8 bar).
The three modes are also reported against the exact global histogram percentile."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1901_03088_amd as s
    return s


@pytest.mark.parametrize("seed,h,w,band_rows", [
    (0, 1024, 1024, 128),     # 8 bands (even count)
    (1, 777, 501, 100),       # 8 bands, last one short, ragged width (unaligned band starts)
    (2, 333, 257, 333),       # one band = the global percentile
    (3, 129, 63, 1),          # one-row bands, odd count
    (4, 50, 7, 3),            # bands of 21 pixels (fewer than 8 aligned units)
])
def test_band_percentiles_match_oracle(S, orc, seed, h, w, band_rows):
    d = synth.make_image(seed, h, w, device=DEV)
    p = S.params()
    W = S.as_basis(d["W"], DEV)
    med, bands, flags = S.spcn_band_percentiles(d["img"], W, band_rows, p)
    torch.cuda.synchronize()
    o_med, o_bp, o_bf, o_f = orc.band_percentiles(d["img"].cpu().numpy(), orc.f32(orc.basis(d["W"])), band_rows,
                                                  lam=orc.f32(p.lambda_))
    assert np.array_equal(bands.cpu().numpy(), o_bp.astype(np.float32))
    assert np.array_equal(med.cpu().numpy(), o_med.astype(np.float32))
    assert (flags.cpu().numpy() & 1).any() == bool(o_f & 1)
    if band_rows >= h:
        _, st = S.spcn_normalize(d["img"], W, W, torch.ones(2, device=DEV), p)
        assert np.array_equal(st["p99_src"].cpu().numpy(), med.cpu().numpy())


def test_band_percentiles_white_bands(S, orc):
    """Bands without tissue are skipped by the median; an all-white image flags NO_TISSUE."""
    d = synth.make_image(6, 256, 256, device=DEV)
    img = d["img"].clone()
    img[64:160] = 250
    W = S.as_basis(d["W"], DEV)
    med, bands, flags = S.spcn_band_percentiles(img, W, 32)
    torch.cuda.synchronize()
    o_med, o_bp, o_bf, _ = orc.band_percentiles(img.cpu().numpy(), orc.f32(orc.basis(d["W"])), 32,
                                                lam=orc.f32(0.01))
    assert np.array_equal(med.cpu().numpy(), o_med.astype(np.float32))
    white = torch.full((64, 64, 3), 250, dtype=torch.uint8, device=DEV)
    med2, _, flags2 = S.spcn_band_percentiles(white, W, 8)
    torch.cuda.synchronize()
    assert med2.cpu().tolist() == [0.0, 0.0] and (flags2.cpu().numpy() & S.FLAG_NO_TISSUE).all()


@pytest.mark.parametrize("seed,h,w,n_s", [(0, 1024, 1024, 20000), (1, 300, 411, 5000), (2, 64, 64, 100000)])
def test_sample_percentile_matches_oracle(S, orc, seed, h, w, n_s):
    d = synth.make_image(seed, h, w, device=DEV)
    p = S.params()
    W = S.as_basis(d["W"], DEV)
    P, flags = S.spcn_sample_percentile(d["img"], W, n_s, seed=99, p=p)
    torch.cuda.synchronize()
    o_P, kept, o_f = orc.sample_percentile(d["img"].cpu().numpy(), orc.f32(orc.basis(d["W"])), n_s, seed=99,
                                           lam=orc.f32(p.lambda_))
    # FP64 on both sides (closed form on the GPU, enumeration in the oracle): equal as FP32 values
    # unless the FP64 results straddle an FP32 rounding boundary (one ulp)
    g = P.cpu().numpy()
    assert np.all(np.abs(g - o_P.astype(np.float32)) <= np.spacing(np.float32(o_P.max()))), (g, o_P)
    assert bool(flags.cpu().numpy()[0] & S.FLAG_SHORT) == (kept < n_s)


@pytest.mark.parametrize("colours", [[(140, 80, 160)], [(140, 80, 160), (90, 60, 150)]])
def test_sample_percentile_ties(S, orc, colours):
    """Samples with many equal densities: one colour (all 40000 samples equal) or two colours in
    halves, so more values share the first two selection digits than the gathering keeps and the
    last digits are taken over all values; the result equals the oracle's nearest rank."""
    h, w = 200, 300
    img = torch.empty((h, w, 3), dtype=torch.uint8, device=DEV)
    for k, c in enumerate(colours):
        img[k * h // len(colours):(k + 1) * h // len(colours)] = torch.tensor(c, dtype=torch.uint8, device=DEV)
    W = synth.reference_basis()
    p = S.params()
    for n_s in (40000, 5000):
        P, flags = S.spcn_sample_percentile(img, S.as_basis(W, DEV), n_s, seed=5, p=p)
        torch.cuda.synchronize()
        o_P, kept, o_f = orc.sample_percentile(img.cpu().numpy(), orc.f32(orc.basis(W)), n_s, seed=5,
                                               lam=orc.f32(p.lambda_))
        g = P.cpu().numpy()
        assert np.all(np.abs(g - o_P.astype(np.float32)) <= np.spacing(np.float32(o_P.max()))), (n_s, g, o_P)
        assert kept == n_s and int(flags.cpu().numpy().max()) == 0


def test_recolor_given_percentiles(S, orc):
    src = synth.make_image(0, 512, 640, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    p = S.params()
    ws, wt = S.as_basis(src["W"], DEV), S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    med, _, _ = S.spcn_band_percentiles(src["img"], ws, 64, p)
    for P in (med, torch.tensor([0.0, 1.3], device=DEV)):
        out, scale, flags = S.spcn_recolor_p99(src["img"], ws, wt, sc, P, p)
        torch.cuda.synchronize()
        o = orc.recolor_u8(src["img"].cpu().numpy(), orc.f32(orc.basis(src["W"])), orc.f32(orc.basis(tgt["W"])),
                           sc.cpu().numpy().astype(np.float64), P.cpu().numpy().astype(np.float64),
                           lam=orc.f32(p.lambda_))
        dd = np.abs(o.astype(int) - out.cpu().numpy().astype(int)).reshape(-1, 3).max(1)
        assert (dd <= 1).mean() >= 0.9999, (dd > 1).sum()
        assert bool(flags.cpu().numpy()[0] & S.FLAG_BIN0) == (float(P[0]) <= 0.0)
    # the global percentile given explicitly reproduces spcn_normalize (up to the FP32 rounding of
    # the reported percentile, which spcn_normalize keeps in FP64)
    out_n, st = S.spcn_normalize(src["img"], ws, wt, sc, p)
    out_g, _, _ = S.spcn_recolor_p99(src["img"], ws, wt, sc, st["p99_src"], p)
    torch.cuda.synchronize()
    diff = (out_n.int() - out_g.int()).abs()
    assert int(diff.max()) <= 1 and float((diff > 0).float().mean()) < 1e-3


def test_modes_against_global_on_config1(S):
    """Report the three percentiles of the 8192^2 image side by side (the paper's modes are
    approximations of the global order statistic; they agree to a few percent on this input)."""
    d = synth.config1(device=DEV)
    p = S.params()
    W = S.as_basis(d["W"], DEV)
    _, st = S.spcn_normalize(d["img"], W, W, torch.ones(2, device=DEV), p)
    med, _, _ = S.spcn_band_percentiles(d["img"], W, 1024, p)
    sp, _ = S.spcn_sample_percentile(d["img"], W, 100000, seed=1, p=p)
    torch.cuda.synchronize()
    g = st["p99_src"].cpu().numpy()
    print(f"\n[modes] global {g} band-median {med.cpu().numpy()} sample {sp.cpu().numpy()}")
    assert np.allclose(med.cpu().numpy(), g, rtol=0.1)
    assert np.allclose(sp.cpu().numpy(), g, rtol=0.1)


def _close32(g, o):
    """FP64 values on both sides (closed form on the GPU, enumeration in the oracle), reported as
    FP32: equal unless the two FP64 results straddle an FP32 rounding boundary (one ulp)."""
    o32 = np.asarray(o).astype(np.float32)
    return np.all(np.abs(np.asarray(g, np.float32) - o32) <= np.spacing(np.maximum(np.abs(o32), np.float32(1e-30))))


@pytest.mark.parametrize("seed,h,w,kw", [
    (0, 1024, 1024, {}),
    (1, 333, 257, {}),                                   # ragged: tail of 1 pixel
    (2, 1, 3, {}),                                       # three pixels, all in the tail
    (3, 50, 7, dict(percentile=50.0)),
    (4, 200, 300, dict(percentile=100.0)),
    (5, 256, 256, dict(hist_hi=(0.25, 0.25))),           # rank k in the overflow bin
    (6, 256, 200, dict(lam=0.0)),
    (7, 128, 128, dict(white_sum=0)),                    # every pixel counts
    (8, 300, 200, dict(hist_hi=(16.0, 16.0), percentile=1.0)),
])
def test_exact_percentile_matches_oracle(S, orc, seed, h, w, kw):
    d = synth.make_image(seed, h, w, device=DEV)
    p = S.params(**kw)
    W = S.as_basis(d["W"], DEV)
    P, flags = S.spcn_exact_percentile(d["img"], W, p)
    torch.cuda.synchronize()
    o_P, n, o_f = orc.exact_percentile(d["img"].cpu().numpy(), orc.f32(orc.basis(d["W"])),
                                       lam=orc.f32(p.lambda_), white_sum=p.white_sum, percentile=p.percentile)
    print(f"\n[exact] seed {seed} {h}x{w} {kw}: n {n} gpu {P.cpu().numpy()} oracle {o_P}")
    assert _close32(P.cpu().numpy(), o_P), (P, o_P)
    assert (flags.cpu().numpy() & S.FLAG_NO_TISSUE).any() == bool(o_f & 1)


def test_exact_percentile_special_images(S, orc):
    """Constant colour (every rank is that colour's density), no tissue, and two calls in a row on
    one workspace (the colour table is cleared by each call)."""
    W = S.as_basis(synth.reference_basis(), DEV)
    Wn = orc.f32(orc.basis(synth.reference_basis()))
    ws = S.workspace(S.workspace_size(S.OP_EXACT_PERCENTILE, 0, 0, 0), DEV)
    col = torch.tensor([140, 80, 160], dtype=torch.uint8, device=DEV).expand(64, 96, 3).contiguous()
    for q in (0.5, 99.0, 100.0):
        P, fl = S.spcn_exact_percentile(col, W, S.params(percentile=q), ws=ws)
        torch.cuda.synchronize()
        Hc, _ = orc.densities_u8(col[:1, :1].cpu().numpy(), Wn)
        assert _close32(P.cpu().numpy(), Hc[:, 0]) and int(fl.cpu().numpy().max()) == 0
    white = torch.full((32, 32, 3), 250, dtype=torch.uint8, device=DEV)
    P, fl = S.spcn_exact_percentile(white, W, ws=ws)
    torch.cuda.synchronize()
    assert P.cpu().tolist() == [0.0, 0.0] and (fl.cpu().numpy() & S.FLAG_NO_TISSUE).all()
    for seed, hw in ((11, (512, 384)), (12, (100, 77))):
        d = synth.make_image(seed, *hw, device=DEV)
        P, _ = S.spcn_exact_percentile(d["img"], S.as_basis(d["W"], DEV), ws=ws)
        torch.cuda.synchronize()
        o_P, _, _ = orc.exact_percentile(d["img"].cpu().numpy(), orc.f32(orc.basis(d["W"])), lam=orc.f32(0.01))
        assert _close32(P.cpu().numpy(), o_P)


def test_exact_percentile_on_config1(S, orc):
    """8192^2 image: the exact order statistic against numpy's selection over the oracle's FP64
    densities of all tissue pixels, and within one bin width of the histogram percentile."""
    d = synth.config1(device=DEV)
    p = S.params()
    W = S.as_basis(d["W"], DEV)
    P, fl = S.spcn_exact_percentile(d["img"], W, p)
    _, st = S.spcn_normalize(d["img"], W, W, torch.ones(2, device=DEV), p)
    torch.cuda.synchronize()
    H, m = orc.densities_u8(d["img"].cpu().numpy(), orc.f32(orc.basis(d["W"])), lam=orc.f32(p.lambda_))
    t = m.astype(bool)
    o_P = np.array([np.percentile(H[j][t], 99, method="inverted_cdf") for j in range(2)])
    del H
    g = P.cpu().numpy()
    print(f"\n[exact] config1: gpu {g} oracle {o_P} histogram {st['p99_src'].cpu().numpy()}")
    assert _close32(g, o_P)
    assert np.all(np.abs(g - st["p99_src"].cpu().numpy()) <= 4.0 / 256)


def test_exact_percentile_list_overflow(S, orc):
    """All 2^24 colours once each with a histogram range of 256 (bins one density unit wide): the
    crossing bins hold more colours than the (key, count) list takes (2^21), so the digit passes scan
    the colour table instead.  At the median both stains overflow (5.9M and 13.8M colours in the
    bin); at q = 90 stain 0 overflows (2.27M) and stain 1 does not (1.64M)."""
    idx = torch.arange(1 << 24, dtype=torch.int64, device=DEV)
    cube = torch.stack([idx & 255, (idx >> 8) & 255, idx >> 16], dim=1).to(torch.uint8).view(4096, 4096, 3)
    W = S.as_basis(synth.reference_basis(), DEV)
    Wn = orc.f32(orc.basis(synth.reference_basis()))
    host = cube.cpu().numpy()
    ws = S.workspace(S.workspace_size(S.OP_EXACT_PERCENTILE, 0, 0, 0), DEV)
    for q in (50.0, 90.0):
        p = S.params(percentile=q, hist_hi=(256.0, 256.0))
        P, fl = S.spcn_exact_percentile(cube, W, p, ws=ws)
        torch.cuda.synchronize()
        o_P, n, o_f = orc.exact_percentile(host, Wn, lam=orc.f32(p.lambda_), percentile=q)
        print(f"[exact overflow q={q}] gpu {P.cpu().numpy()} oracle {o_P} (n = {n})", flush=True)
        assert _close32(P.cpu().numpy(), o_P)
        assert int(fl.cpu().numpy().max()) == 0
