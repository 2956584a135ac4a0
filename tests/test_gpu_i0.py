"""GPU parity of the channel-wise background intensity (Sec. 3.1 item 1) with the FP64 oracle:
identical integer estimates and flags (the decisions are integer: the same draws, the same
threshold, the same nearest rank), and normalisation with estimated i0 against the oracle run with
the same i0."""
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


@pytest.mark.parametrize("seed,h,w,n_s,bg,q", [
    (0, 1024, 1024, 100000, 0.3, 80.0),
    (3, 333, 517, 5000, 0.3, 80.0),
    (4, 200, 300, 20000, 0.05, 80.0),      # few background pixels: short sample
    (5, 256, 256, 1, 0.5, 80.0),
    (6, 512, 384, 30000, 0.4, 100.0),
    (7, 512, 384, 30000, 0.4, 0.5),
])
def test_i0_matches_oracle(S, orc, seed, h, w, n_s, bg, q):
    d = synth.make_image(seed, h, w, bg_frac=bg, device=DEV)
    i0, flags = S.spcn_estimate_i0(d["img"], n_s, seed=1000 + seed, percentile=q)
    torch.cuda.synchronize()
    o_i0, kept = orc.estimate_i0(d["img"].cpu().numpy(), n_s, seed=1000 + seed, percentile=q)
    assert np.array_equal(i0.cpu().numpy().astype(np.float64), o_i0), (i0, o_i0)
    f = int(flags.cpu()[0])
    assert bool(f & S.FLAG_SHORT) == (kept < n_s)
    assert not (f & S.FLAG_NO_BACKGROUND)


def test_i0_no_background(S):
    img = torch.full((64, 64, 3), 100, dtype=torch.uint8, device=DEV)
    i0, flags = S.spcn_estimate_i0(img, 1000, seed=1)
    torch.cuda.synchronize()
    assert i0.cpu().tolist() == [255.0, 255.0, 255.0]
    assert int(flags.cpu()[0]) & S.FLAG_NO_BACKGROUND


def test_i0_config1_size(S, orc):
    d = synth.config1(device=DEV)
    i0, _ = S.spcn_estimate_i0(d["img"], 100000, seed=5)
    torch.cuda.synchronize()
    o_i0, _ = orc.estimate_i0(d["img"].cpu().numpy(), 100000, seed=5)
    assert np.array_equal(i0.cpu().numpy().astype(np.float64), o_i0)


def test_normalize_with_estimated_i0(S, orc):
    """The estimates feed Eq. 1 (source i0) and Eq. 4 (target's i0 as i0_out); the uint8 output
    matches the oracle run with the same i0 at the usual bar."""
    src = synth.make_image(0, 512, 640, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    i0s, _ = S.spcn_estimate_i0(src["img"], 50000, seed=11)
    i0t, _ = S.spcn_estimate_i0(tgt["img"], 50000, seed=12)
    i0s_h = i0s.cpu().numpy().astype(np.float64)
    i0t_h = i0t.cpu().numpy().astype(np.float64)
    ws, wt = S.as_basis(src["W"], DEV), S.as_basis(tgt["W"], DEV)
    pt = S.params(i0=tuple(i0t_h))
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, pt, want_h=False)
    ps = S.params(i0=tuple(i0s_h))
    out, st = S.spcn_normalize(src["img"], ws, wt, sc, ps, i0_out=tuple(i0t_h))
    torch.cuda.synchronize()
    o_out, o_st, _ = orc.normalize_u8(src["img"].cpu().numpy(), orc.f32(orc.basis(src["W"])),
                                       orc.f32(orc.basis(tgt["W"])), sc.cpu().numpy().astype(np.float64),
                                       i0_in=i0s_h, i0_out=i0t_h, lam=orc.f32(ps.lambda_))
    dd = np.abs(o_out.astype(int) - out.cpu().numpy().astype(int)).reshape(-1, 3).max(1)
    assert (dd <= 1).mean() >= 0.9999, (dd > 1).sum()
    assert np.array_equal(o_st["P"].astype(np.float32), st["p99_src"].cpu().numpy())
