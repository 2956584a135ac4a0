"""GPU parity of the uint8 path (spcn_densities, spcn_normalize) against the FP64 oracle.

Bars: histogram counts bit-exact; densities within 1e-4 * max(|h|, 1); output within one uint8
level on >= 99.99% of pixels (mismatch counts printed); percentiles equal (same counts, same FP64
formula).  Inputs are seeded synthetic images; the oracle always receives the very tensor the GPU
received, copied to the host.
"""
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


def np_img(t):
    return t.detach().cpu().numpy()


def gpu_densities(S, img, W, p):
    w = S.as_basis(W, DEV)
    h, hist, p99, flags = S.spcn_densities(img, w, p)
    torch.cuda.synchronize()
    return h.cpu().numpy().astype(np.float64), hist.cpu().numpy().astype(np.uint64), p99.cpu().numpy(), flags.cpu().numpy()


def oracle_densities(orc, img, W, p):
    """The oracle's densities, histogram, percentile and flags; with p.auto_range the histogram is
    over the oracle's settled ranges (one doubling of a stain whose percentile lands in the last bin)."""
    i0 = list(p.i0)
    H, m = orc.densities_u8(np_img(img), orc.f32(orc.basis(W)), i0, orc.f32(p.lambda_), p.white_sum)
    hh, bits = list(p.hist_hi), 0
    if p.auto_range:
        hh, bits = orc.settle_range(H, m, hh, p.percentile)
    hist = orc.histogram(H, m, hh, 256)
    P = []
    fl = []
    for j in range(2):
        Pj, f, _ = orc.percentile_hist(hist[j], float(hh[j]), orc.q_of(p.percentile))
        P.append(Pj); fl.append(f | (orc.RANGE_RETRY if bits >> j & 1 else 0))
    return H, m, hist, np.array(P), np.array(fl)


def report(tag, a, b):
    d = np.abs(a.astype(np.int32) - b.astype(np.int32))
    n = d.size // 3
    px = d.reshape(-1, 3).max(axis=1)
    print(f"[{tag}] pixels={n} exact={int((px == 0).sum())} off_by_1={int((px == 1).sum())} worse={int((px > 1).sum())}",
          flush=True)
    return px


# ------------------------------------------------------------------ densities and histogram

@pytest.mark.parametrize("lam", [0.01, 0.1, 0.0])
def test_densities_config0(S, orc, lam):
    d = synth.make_image(0, 1024, 1024, device=DEV)
    p = S.params(lam=lam)
    h, hist, p99, flags = gpu_densities(S, d["img"], d["W"], p)
    H, m, ohist, P, fl = oracle_densities(orc, d["img"], d["W"], p)
    assert np.array_equal(hist, ohist), "histogram counts differ"
    err = np.abs(h - H) / np.maximum(np.abs(H), 1.0)
    print(f"[densities lam={lam}] max rel err {err.max():.3e}", flush=True)
    assert err.max() <= 1e-4
    assert np.array_equal(p99, P.astype(np.float32))
    assert np.array_equal(flags, fl)


@pytest.mark.parametrize("shape", [(1, 1), (1, 3), (3, 5), (37, 53), (64, 64), (129, 257), (1000, 7)])
def test_densities_ragged_shapes(S, orc, shape):
    d = synth.make_image(7 + shape[0], shape[0], shape[1], device=DEV)
    p = S.params()
    h, hist, p99, flags = gpu_densities(S, d["img"], d["W"], p)
    H, m, ohist, P, fl = oracle_densities(orc, d["img"], d["W"], p)
    assert np.array_equal(hist, ohist)
    assert np.abs(h - H).max() <= 1e-4 * max(1.0, np.abs(H).max())
    assert np.array_equal(p99, P.astype(np.float32))


def rgb_cube():
    v = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([v & 255, (v >> 8) & 255, v >> 16], axis=-1).astype(np.uint8)
    return img.reshape(4096, 4096, 3)


@pytest.mark.parametrize("case", ["cfg0", "reference", "wide", "lam0", "lam01_hi8", "nomask_hi1"])
def test_histogram_exhaustive_rgb_cube(S, orc, case):
    """Every 8-bit RGB triple once: equal counts for all 2^24 pixels prove equal bins for every
    image with this basis (density is a function of the triple alone)."""
    cube = rgb_cube()
    W = {"cfg0": synth.make_image(0, 8, 8)["W"], "reference": synth.reference_basis(),
         "wide": synth.jitter_basis(np.random.default_rng(5), 20.0),
         "lam0": synth.make_image(1, 8, 8)["W"], "lam01_hi8": synth.make_image(2, 8, 8)["W"],
         "nomask_hi1": synth.make_image(3, 8, 8)["W"]}[case]
    p = S.params(auto_range=False)      # bins at the given range, whatever the percentile
    if case == "lam0":
        p = S.params(lam=0.0, auto_range=False)
    if case == "lam01_hi8":
        p = S.params(lam=0.1, hist_hi=(8.0, 2.0), auto_range=False)
    if case == "nomask_hi1":
        p = S.params(white_sum=0, hist_hi=(1.0, 0.5), auto_range=False)
    img = torch.from_numpy(cube).to(DEV)
    w = S.as_basis(W, DEV)
    H, m = orc.densities_u8(cube, orc.f32(orc.basis(W)), list(p.i0), orc.f32(p.lambda_), p.white_sum)
    ohist = orc.histogram(H, m, list(p.hist_hi), 256)
    saved = S.get_option(S.OPT_P1_VARIANT)
    try:
        for v in range(10):   # every pass-1 layout and tile order (the cube spans many tiles of each)
            S.set_option(S.OPT_P1_VARIANT, v)
            _, hist, p99, _ = S.spcn_densities(img, w, p, want_h=False)
            torch.cuda.synchronize()
            ghist = hist.cpu().numpy().astype(np.uint64)
            diff = (ghist.astype(np.int64) - ohist.astype(np.int64))
            print(f"[cube {case} variant {v}] total={int(ohist.sum())} abs diff sum={int(np.abs(diff).sum())}",
                  flush=True)
            assert np.array_equal(ghist, ohist), v
    finally:
        S.set_option(S.OPT_P1_VARIANT, saved)


# ------------------------------------------------------------------ fused normalisation

def run_normalize(S, src_img, Ws, tgt_img, Wt, p, i0_out=None):
    wt = S.as_basis(Wt, DEV)
    _, _, scale_tgt, _ = S.spcn_densities(tgt_img, wt, p, want_h=False)
    out, st = S.spcn_normalize(src_img, S.as_basis(Ws, DEV), wt, scale_tgt, p, i0_out=i0_out)
    torch.cuda.synchronize()
    return out, {k: v.cpu().numpy() for k, v in st.items()}, scale_tgt.cpu().numpy()


def oracle_normalize(orc, src, Ws, Wt, scale_tgt, p, i0_out=None):
    return orc.normalize_u8(np_img(src), orc.f32(orc.basis(Ws)), orc.f32(orc.basis(Wt)),
                            scale_tgt.astype(np.float64), list(p.i0), list(i0_out or p.i0),
                            orc.f32(p.lambda_), p.white_sum, p.percentile, list(p.hist_hi), 256,
                            auto_range=bool(p.auto_range))


def check_normalize(tag, out, st, o_out, o_st, o_hist):
    assert np.array_equal(st["hist"].astype(np.uint64), o_hist)
    assert np.array_equal(st["p99_src"], o_st["P"].astype(np.float32))
    assert np.array_equal(st["flags"], o_st["flags"])
    assert np.allclose(st["scale"], o_st["scale"], rtol=1e-7)
    px = report(tag, np_img(out), o_out)
    assert (px <= 1).mean() >= 0.9999
    # FP32 vs FP64 rounding can only flip values within ~1e-3 level of a half-level boundary
    assert (px == 0).mean() >= 0.98


def test_normalize_config0(S, orc):
    src = synth.make_image(0, 1024, 1024, device=DEV)
    tgt = synth.make_image(1, 1024, 1024, device=DEV)
    p = S.params()
    out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p)
    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, p)
    check_normalize("cfg0", out, st, o_out, o_st, o_hist)


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (37, 53), (255, 257), (512, 1000)])
def test_normalize_ragged(S, orc, shape):
    src = synth.make_image(100 + shape[1], shape[0], shape[1], device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    p = S.params()
    out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p, i0_out=(250.0, 245.0, 240.0))
    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, p, i0_out=(250.0, 245.0, 240.0))
    check_normalize(f"ragged{shape}", out, st, o_out, o_st, o_hist)


def test_normalize_all_white(S, orc):
    img = torch.full((40, 40, 3), 250, dtype=torch.uint8, device=DEV)
    tgt = synth.make_image(1, 128, 128, device=DEV)
    p = S.params()
    out, st, sc = run_normalize(S, img, synth.reference_basis(), tgt["img"], tgt["W"], p)
    assert (st["flags"] & S.FLAG_NO_TISSUE).all()
    assert np.array_equal(st["scale"], [1.0, 1.0])
    o_out, o_st, o_hist = oracle_normalize(orc, img, synth.reference_basis(), tgt["W"], sc, p)
    check_normalize("white", out, st, o_out, o_st, o_hist)


def test_normalize_range_flag(S, orc):
    """hist_hi far below the densities and no automatic retry: the percentile lands in the overflow
    bin and the flag says so."""
    src = synth.make_image(5, 200, 200, device=DEV)
    tgt = synth.make_image(1, 200, 200, device=DEV)
    p = S.params(hist_hi=(0.125, 0.125), auto_range=False)
    out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p)
    assert (st["flags"] & S.FLAG_RANGE).all(), st["flags"]
    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, p)
    check_normalize("range", out, st, o_out, o_st, o_hist)


def overflowing_ranges(orc, img, W, p):
    """Per stain, the power of two just below the exact percentile (P in [r, 2r)): the histogram
    percentile at r falls in the open last bin, at 2r inside the range."""
    H, m = orc.densities_u8(np_img(img), orc.f32(orc.basis(W)), list(p.i0), orc.f32(p.lambda_), p.white_sum)
    P = [orc.percentile_exact(H[j], m, orc.q_of(p.percentile))[0] for j in range(2)]
    return [2.0 ** np.floor(np.log2(Pj)) for Pj in P]


@pytest.mark.parametrize("stains", [(0,), (1,), (0, 1)])
def test_normalize_range_retry(S, orc, stains):
    """A range that the percentile overflows: pass 1 is repeated on the device at twice that
    stain's range (the other stain keeps its range), and every result equals the oracle's at the
    doubled range; the flags report the retry and no overflow."""
    src = synth.make_image(5, 300, 200, device=DEV)
    tgt = synth.make_image(1, 200, 200, device=DEV)
    r = overflowing_ranges(orc, src["img"], src["W"], S.params())
    given = [r[j] if j in stains else 4.0 * r[j] for j in range(2)]
    used = [2.0 * r[j] if j in stains else 4.0 * r[j] for j in range(2)]
    out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], S.params(hist_hi=given))
    assert list(st["hist_hi"]) == used
    # the oracle settles the same range from the given one and reports the same retry bits
    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, S.params(hist_hi=given))
    assert o_st["hist_hi"] == used
    check_normalize("retry", out, st, o_out, o_st, o_hist)
    assert [bool(f & S.FLAG_RANGE_RETRY) for f in st["flags"]] == [j in stains for j in range(2)]
    # without the retry: the oracle at the given range, overflow flagged
    p0 = S.params(hist_hi=given, auto_range=False)
    out0, st0, sc0 = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p0)
    o_out0, o_st0, o_hist0 = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc0, p0)
    check_normalize("no retry", out0, st0, o_out0, o_st0, o_hist0)
    assert [bool(f & S.FLAG_RANGE) for f in st0["flags"]] == [j in stains for j in range(2)]


def test_densities_range_retry_and_recolor(S, orc):
    """spcn_densities repeats pass 1 the same way and reports the range; spcn_recolor from that
    histogram and range equals spcn_normalize byte for byte."""
    src = synth.make_image(9, 256, 320, device=DEV)
    tgt = synth.make_image(1, 200, 200, device=DEV)
    r = overflowing_ranges(orc, src["img"], src["W"], S.params())
    p = S.params(hist_hi=(r[0], 4.0 * r[1]))
    w = S.as_basis(src["W"], DEV)
    hh = torch.empty(2, dtype=torch.float32, device=DEV)
    _, hist, p99, flags = S.spcn_densities(src["img"], w, p, want_h=False, hist_hi_out=hh)
    torch.cuda.synchronize()
    assert hh.cpu().tolist() == [2.0 * r[0], 4.0 * r[1]]
    H, m, ohist, P, fl = oracle_densities(orc, src["img"], src["W"], S.params(hist_hi=hh.cpu().tolist()))
    assert np.array_equal(hist.cpu().numpy().astype(np.uint64), ohist)
    assert np.array_equal(p99.cpu().numpy(), P.astype(np.float32))
    assert list(flags.cpu().numpy()) == [fl[0] | S.FLAG_RANGE_RETRY, fl[1]]
    wt = S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, S.params(), want_h=False)
    ref, _ = S.spcn_normalize(src["img"], w, wt, sc, p)
    out, st = S.spcn_recolor(src["img"], w, wt, sc, hist, S.params(hist_hi_dev=hh))
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert st["hist_hi"].cpu().tolist() == hh.cpu().tolist()


def test_range_from_basis_sample(S, orc):
    """spcn_estimate_basis derives the range from its sample percentile (the power of two at or
    above twice it, within [2^-4, 2^6]); a normalisation that reads it from the device equals the
    oracle's at that range, with no overflow."""
    import math
    src = synth.make_image(0, 1024, 1024, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    hh = torch.empty(2, dtype=torch.float32, device=DEV)
    w, sp, _ = S.spcn_estimate_basis(src["img"], 20000, seed=3, p=S.params(), hist_hi_out=hh)
    torch.cuda.synchronize()
    for j in range(2):
        v = 2.0 * float(sp[j])
        m_, e_ = math.frexp(v)
        want = 0.0625 if v <= 0.0625 else 64.0 if v >= 64.0 else (v if m_ == 0.5 else 2.0 ** e_)
        assert float(hh[j]) == want, (j, float(hh[j]), want)
    p = S.params(hist_hi_dev=hh)
    wt = S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, S.params(), want_h=False)
    out, st = S.spcn_normalize(src["img"], w, wt, sc, p)
    torch.cuda.synchronize()
    stn = {k: v.cpu().numpy() for k, v in st.items()}
    assert stn["hist_hi"].tolist() == hh.cpu().tolist()
    assert not (stn["flags"] & (S.FLAG_RANGE | S.FLAG_RANGE_RETRY)).any()
    Wf = w.cpu().numpy().astype(np.float64)
    o_out, o_st, o_hist = orc.normalize_u8(np_img(src["img"]), Wf, orc.f32(orc.basis(tgt["W"])),
                                           sc.cpu().numpy().astype(np.float64), lam=orc.f32(0.01),
                                           hist_hi=hh.cpu().numpy().astype(np.float64).tolist())
    check_normalize("range from sample", out, stn, o_out, o_st, o_hist)


def test_normalize_graph_replay_with_retry(S):
    """spcn_normalize with a range that triggers the device-side retry, captured in a graph and
    replayed with eager work in between: every replay equals the eager result."""
    src = synth.make_image(5, 300, 200, device=DEV)
    tgt = synth.make_image(1, 200, 200, device=DEV)
    wt = S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, S.params(), want_h=False)
    ws = S.as_basis(src["W"], DEV)
    p = S.params(hist_hi=(0.5, 0.5))
    ref, st_ref = S.spcn_normalize(src["img"], ws, wt, sc, p)
    torch.cuda.synchronize()
    assert (st_ref["flags"].cpu() & S.FLAG_RANGE_RETRY).any()
    out = torch.empty_like(src["img"])
    wsp = S.workspace(S.workspace_size(S.OP_NORMALIZE), DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        S.spcn_normalize(src["img"], ws, wt, sc, p, out=out, stats=False, ws=wsp)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        S.spcn_normalize(src["img"], ws, wt, sc, p, out=out, stats=False, ws=wsp)
    for k in range(3):
        out.zero_()
        S.spcn_normalize(tgt["img"], wt, wt, sc, S.params(), out=torch.empty_like(tgt["img"]))   # eager work between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k


def test_normalize_bin0_flag(S, orc):
    """A pale flat tissue image with a wide histogram: the percentile lands in bin 0 and the
    scale stays 1."""
    img = torch.full((64, 64, 3), 215, dtype=torch.uint8, device=DEV)
    tgt = synth.make_image(1, 200, 200, device=DEV)
    p = S.params(hist_hi=(256.0, 256.0))
    out, st, sc = run_normalize(S, img, synth.reference_basis(), tgt["img"], tgt["W"], p)
    assert (st["flags"] & S.FLAG_BIN0).all(), st["flags"]
    assert np.array_equal(st["scale"], [1.0, 1.0])
    o_out, o_st, o_hist = oracle_normalize(orc, img, synth.reference_basis(), tgt["W"], sc, p)
    check_normalize("bin0", out, st, o_out, o_st, o_hist)


def test_normalize_identity_on_target(S, orc):
    """Normalising the target with its own basis and percentiles: every scale is exactly 1."""
    tgt = synth.make_image(1, 512, 512, device=DEV)
    p = S.params()
    out, st, sc = run_normalize(S, tgt["img"], tgt["W"], tgt["img"], tgt["W"], p)
    assert np.array_equal(st["scale"], [1.0, 1.0])
    o_out, o_st, o_hist = oracle_normalize(orc, tgt["img"], tgt["W"], tgt["W"], sc, p)
    check_normalize("identity", out, st, o_out, o_st, o_hist)


def test_degenerate_basis_flag(S):
    img = synth.make_image(3, 64, 64, device=DEV)["img"]
    W = np.array([[0.6, 0.6], [0.7, 0.7], [0.3, 0.3]])     # parallel columns: singular Gram matrix
    h, hist, p99, flags = gpu_densities(S, img, W, S.params())
    assert (flags & S.FLAG_BASIS).all()
    assert (h == 0).all()


@pytest.mark.parametrize("W", [
    [[0.65, -0.05], [0.70, 0.99], [0.29, 0.11]],    # a negative entry with a positive Gram cross term
    [[0.9, -0.3], [0.1, 0.9], [0.4, 0.3]],          # negative cross term g01 < 0
    [[0.65, 0.07], [float("nan"), 0.99], [0.29, 0.11]],   # a NaN entry
    [[0.65, 0.07], [0.70, float("inf")], [0.29, 0.11]],   # an infinite entry
])
def test_negative_basis_refused(S, W):
    """Eq. 2 requires W >= 0 (the closed-form density solve relies on it): a basis with a negative
    or non-finite entry is refused on the device -- SPCN_FLAG_BASIS, every density 0, the
    normalisation leaves every pixel unscaled -- instead of returning densities of another problem."""
    img = synth.make_image(4, 64, 96, device=DEV)["img"]
    W = np.array(W)
    h, hist, p99, flags = gpu_densities(S, img, W, S.params())
    assert (flags & S.FLAG_BASIS).all()
    assert (h == 0).all()
    tgt = synth.make_image(1, 64, 64, device=DEV)
    out, st = S.spcn_normalize(img, S.as_basis(W, DEV), S.as_basis(tgt["W"], DEV),
                               torch.tensor([1.0, 1.0], device=DEV), S.params())
    torch.cuda.synchronize()
    assert (st["flags"].cpu().numpy() & S.FLAG_BASIS).all()


@pytest.mark.parametrize("bad", [(float("nan"), float("inf")), (-1.0, 0.0)])
def test_invalid_target_scale_refused(S, orc, bad):
    """A target scale that is not finite and positive is refused per stain (SPCN_FLAG_SCALE) and the
    stain keeps scale 1: the output is the oracle's recolouring with s = 1 (its target scale set to
    the source percentile), the histogram and percentile as usual; the batched path flags the same."""
    src = synth.make_image(0, 512, 512, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    p = S.params()
    ws, wt = S.as_basis(src["W"], DEV), S.as_basis(tgt["W"], DEV)
    sc = torch.tensor(bad, dtype=torch.float32, device=DEV)
    out, st = S.spcn_normalize(src["img"], ws, wt, sc, p)
    torch.cuda.synchronize()
    st = {k: v.cpu().numpy() for k, v in st.items()}
    _, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], np.ones(2), p)
    assert np.array_equal(st["hist"].astype(np.uint64), o_hist)
    assert np.array_equal(st["p99_src"], o_st["P"].astype(np.float32))
    assert np.array_equal(st["flags"], o_st["flags"] | S.FLAG_SCALE)
    assert (st["scale"] == 1.0).all()
    P = np.asarray(o_st["P"], dtype=np.float64)
    o = orc.recolor_u8(np_img(src["img"]), orc.f32(orc.basis(src["W"])), orc.f32(orc.basis(tgt["W"])), P, P,
                       lam=orc.f32(p.lambda_))
    px = report("scale refused", np_img(out), o)
    assert (px <= 1).all()
    assert (px == 0).mean() >= 0.98
    tiles = [src["img"], tgt["img"]]
    outs = [torch.empty_like(t) for t in tiles]
    Wb = torch.stack([ws, S.as_basis(tgt["W"], DEV)])
    bs = S.spcn_normalize_batched(S.tile_table(tiles, outs), 2, sum(t.shape[0] * t.shape[1] for t in tiles), Wb, wt,
                                  sc, p)
    torch.cuda.synchronize()
    assert (bs["flags"].cpu().numpy() & S.FLAG_SCALE).all()
    assert (bs["scale"].cpu().numpy() == 1.0).all()


def test_config1_densities_full_size(S, orc):
    """8192 x 8192 (67 Mpixel): spcn_densities with the FP32 density planes, in the benchmark's launch
    shape (the fused pass 1); every density of both planes within 1e-4 max(|h|, 1) of the oracle's
    FP64 value and within the header's bound 2e-6 max(1, hist_hi), the histogram bit-exact,
    percentile and flags equal."""
    src = synth.config1(device=DEV)
    p = S.params()
    h, hist, p99, flags = gpu_densities(S, src["img"], src["W"], p)
    H, m, ohist, P, fl = oracle_densities(orc, src["img"], src["W"], p)
    assert np.array_equal(hist, ohist), "histogram counts differ"
    err = np.abs(h - H) / np.maximum(np.abs(H), 1.0)
    print(f"[cfg1 densities] max rel err {err.max():.3e}, max abs err {np.abs(h - H).max():.3e} over {H.size} values",
          flush=True)
    assert err.max() <= 1e-4
    assert np.abs(h - H).max() <= 2e-6 * max(1.0, max(float(v) for v in p.hist_hi))
    assert np.array_equal(p99, P.astype(np.float32))
    assert np.array_equal(flags, fl)


@pytest.mark.parametrize("shape", [(4, 4), (2, 7), (5, 5), (3, 1)])
def test_densities_plane_alignment(S, orc, shape):
    """Pixel counts that are not a multiple of 4 (the second plane starts off a 16-byte boundary) and
    a tail after the last unit: every density lands at its index, nothing is written past the planes."""
    d = synth.make_image(60 + shape[1], shape[0], shape[1], device=DEV)
    n = shape[0] * shape[1]
    p = S.params()
    w = S.as_basis(d["W"], DEV)
    guard = torch.full((2 * n + 64,), -7.0, dtype=torch.float32, device=DEV)
    h_out = guard[:2 * n]
    _, hist, _, _ = S.spcn_densities(d["img"], w, p, h_out=h_out)
    torch.cuda.synchronize()
    H, m, ohist, P, fl = oracle_densities(orc, d["img"], d["W"], p)
    g = h_out.cpu().numpy().astype(np.float64).reshape(2, n)
    assert np.abs(g - H).max() <= 1e-4 * max(1.0, np.abs(H).max())
    assert np.abs(g - H).max() <= 2e-6 * max(1.0, max(float(v) for v in p.hist_hi))
    assert (guard[2 * n:].cpu().numpy() == -7.0).all()
    assert np.array_equal(hist.cpu().numpy().astype(np.uint64), ohist)


def test_config1_full_size(S, orc):
    """8192 x 8192 (67 Mpixel), the fused path at its benchmark launch shape: full histogram and
    output compared with the oracle."""
    src = synth.config1(device=DEV)
    tgt = synth.target_image(device=DEV)
    p = S.params()
    out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p)
    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, p)
    check_normalize("cfg1", out, st, o_out, o_st, o_hist)


def test_kernel_variants_identical(S, orc):
    """Every tuning variant (table copies, histogram columns, workgroups per CU) gives the same
    histogram, statistics and output bytes."""
    src = synth.make_image(0, 700, 900, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    p = S.params()
    saved = [S.get_option(o) for o in range(4)]
    ref = None
    try:
        for v1 in range(10):
            for v2, bpc in ((0, 8), (1, 4), (2, 1), (0, 2), (3, 2), (4, 1), (5, 1)):
                S.set_option(S.OPT_P1_VARIANT, v1)
                S.set_option(S.OPT_P2_VARIANT, v2)
                S.set_option(S.OPT_P2_BLOCKS_PER_CU, bpc)
                out, st, sc = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p)
                cur = (out.cpu().numpy(), st["hist"], st["p99_src"], st["scale"])
                if ref is None:
                    ref = cur
                    o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc, p)
                    check_normalize("variants", out, st, o_out, o_st, o_hist)
                else:
                    for a, b in zip(ref, cur):
                        assert np.array_equal(a, b), (v1, v2, bpc)
    finally:
        for o, v in enumerate(saved):
            S.set_option(o, v)


def test_option_validation(S):
    import ctypes
    assert S._L.spcn_set_option(0, 10) == S.SPCN_E_ARG
    assert S._L.spcn_set_option(7, 0) == S.SPCN_E_ARG
    assert S.get_option(7) == -1


def test_autotune_image_sets_a_measured_choice(S, orc):
    """The tuner times every pass-1 and pass-2 variant on a 1024^2 image (identical bytes required,
    else it raises), re-times its finalists, leaves the winner set and reports every timing; the
    normalisation under the chosen options still matches the oracle."""
    from paper_1901_03088_amd import autotune
    src = synth.make_image(0, 1024, 1024, device=DEV)
    tgt = synth.make_image(1, 1024, 1024, device=DEV)
    p = S.params()
    ws, wt = S.as_basis(src["W"], DEV), S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    saved = autotune.current()
    try:
        res = autotune.tune_image(src["img"], ws, wt, sc, p, reps=3)
        cur = autotune.current()
        for k in ("p1_variant", "p2_variant", "p2_blocks_per_cu"):
            assert cur[k] == res["options"][k], k
        assert len(res["pass1"]) == len(autotune.P1_CANDIDATES) and len(res["pass2"]) == len(autotune.P2_CANDIDATES)
        assert sum("final_ms" in r for r in res["pass1"]) == 3 and sum("final_ms" in r for r in res["pass2"]) == 3
        out, st, sc2 = run_normalize(S, src["img"], src["W"], tgt["img"], tgt["W"], p)
        o_out, o_st, o_hist = oracle_normalize(orc, src["img"], src["W"], tgt["W"], sc2, p)
        check_normalize("autotuned", out, st, o_out, o_st, o_hist)
    finally:
        autotune.apply(saved)


def test_bandwidth_probe(S):
    """The bandwidth reference kernels: the copy reproduces its source byte for byte (ragged tail of
    the last tile included), the read pass runs and leaves its source untouched."""
    g = torch.Generator(device=DEV)
    g.manual_seed(3)
    src = torch.randint(0, 256, ((1 << 22) + 48,), dtype=torch.uint8, device=DEV, generator=g)
    keep = src.clone()
    for copy_mode, read_mode in ((0, 1), (2, 3)):     # streaming and default cache policy
        dst = torch.zeros_like(src)
        S.spcn_bandwidth_probe(src, dst, copy_mode)
        S.spcn_bandwidth_probe(src, None, read_mode)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), copy_mode
        assert torch.equal(src, keep), read_mode
