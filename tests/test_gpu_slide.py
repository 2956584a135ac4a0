"""Full-size parity on the 50000 x 40000 (2 Gpixel) slide, in the launch configuration the benchmark
times (the default kernel variants, which are the ones the autotuner picks there).

* Histogram counts bit-exact against the oracle, whose histogram is assembled slot by slot from
  the slide's own pixels (every slot is a field of its own seed).
* Percentile and scale equal to the oracle's (same counts, same FP64 formula).
* Every output pixel against the oracle's recolouring of the slide (band by band, the differences
  counted on the device): all within one uint8 level, at most 0.1% off by one.
* The basis fitted from 200k samples of the slide against the oracle's fit on the same samples.
"""
import math

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


@pytest.fixture(scope="module")
def slide():
    img, W, plan = synth.make_slide(device=DEV)
    torch.cuda.synchronize()
    return {"img": img, "W": W, "plan": plan}


def oracle_slide_hist(orc, slide, Wn, p):
    """The oracle's histogram of the whole slide, slot by slot (the GPU's input, copied to the host)."""
    total = np.zeros((2, 256), dtype=np.uint64)
    for y0, x0, hh, ww, _ in slide["plan"]:
        px = slide["img"][y0:y0 + hh, x0:x0 + ww].cpu().numpy()
        H, m = orc.densities_u8(px, Wn, list(p.i0), orc.f32(p.lambda_), p.white_sum)
        total += orc.histogram(H, m, list(p.hist_hi), 256)
        del H, m
    return total


def test_slide_normalize_full_size(S, orc, slide):
    img = slide["img"]
    p = S.params()
    tgt = synth.target_image(device=DEV)
    ws, wt = S.as_basis(slide["W"], DEV), S.as_basis(tgt["W"], DEV)
    _, _, scale_tgt, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    out, st = S.spcn_normalize(img, ws, wt, scale_tgt, p)
    torch.cuda.synchronize()
    ghist = st["hist"].cpu().numpy().astype(np.uint64)
    Wn, Wtn = orc.f32(orc.basis(slide["W"])), orc.f32(orc.basis(tgt["W"]))
    ohist = oracle_slide_hist(orc, slide, Wn, p)
    n = int(ohist[0].sum())
    print(f"\n[slide] tissue pixels {n} ({n / (synth.SLIDE_H * synth.SLIDE_W):.3f}); "
          f"abs count diff {int(np.abs(ghist.astype(np.int64) - ohist.astype(np.int64)).sum())}", flush=True)
    assert np.array_equal(ghist, ohist)
    P = []
    for j in range(2):
        Pj, f, _ = orc.percentile_hist(ohist[j], float(p.hist_hi[j]), orc.q_of(p.percentile))
        assert f == 0
        P.append(Pj)
    P = np.array(P)
    sc = scale_tgt.cpu().numpy().astype(np.float64)
    assert np.array_equal(st["p99_src"].cpu().numpy(), P.astype(np.float32))
    assert np.allclose(st["scale"].cpu().numpy(), sc / P, rtol=1e-7)
    assert (st["flags"].cpu().numpy() == 0).all()
    # every output pixel: the oracle recolours the slide band by band (its OpenMP loops), and the
    # per-pixel largest channel difference is counted on the device
    rows = 2500
    n_exact = n_one = n_worse = worst = 0
    for r0 in range(0, synth.SLIDE_H, rows):
        o = orc.recolor_u8(img[r0:r0 + rows].cpu().numpy(), Wn, Wtn, sc, P, lam=orc.f32(p.lambda_))
        d = (torch.from_numpy(o).to(DEV).to(torch.int16) - out[r0:r0 + rows].to(torch.int16)).abs().amax(dim=2)
        n_exact += int((d == 0).sum()); n_one += int((d == 1).sum()); n_worse += int((d > 1).sum())
        worst = max(worst, int(d.max()))
        del o, d
    n_all = synth.SLIDE_H * synth.SLIDE_W
    print(f"[slide] every output pixel ({n_all}): exact {n_exact} off by 1 {n_one} worse {n_worse} "
          f"(largest difference {worst})", flush=True)
    assert n_exact + n_one + n_worse == n_all
    assert n_worse == 0                      # every pixel within one level (measured: 1.8e5 off by one)
    assert n_one / n_all <= 1e-3


def test_slide_basis_full_size(S, orc, slide):
    img = slide["img"]
    p = S.params()
    w, sp, flags = S.spcn_estimate_basis(img, 200000, seed=2024, p=p, lambda_nmf=0.1, n_iter=50)
    torch.cuda.synchronize()
    host = img.cpu().numpy()
    idx = orc.sample_tissue(host, 200000, 2024, p.white_sum)
    V = orc.od_samples(host, idx, list(p.i0))
    del host
    H0 = np.array([0.65, 0.70, 0.29]); E0 = np.array([0.07, 0.99, 0.11])
    W_init = orc.f32(np.stack([H0 / np.linalg.norm(H0), E0 / np.linalg.norm(E0)], axis=1))
    Wo, spo, _ = orc.nmf(V, orc.f32(0.1), 50, W_init, p.percentile)
    a = np.asarray(w.cpu().numpy(), np.float64).reshape(2, 3)
    b = np.asarray(Wo, np.float64).reshape(2, 3)
    ang = [math.acos(min(1.0, a[j] @ b[j] / (np.linalg.norm(a[j]) * np.linalg.norm(b[j])))) for j in range(2)]
    print(f"\n[slide basis] angle rad {ang}, p99 gpu {sp.cpu().numpy()} oracle {spo}", flush=True)
    assert max(ang) < 1e-6
    assert np.allclose(sp.cpu().numpy(), spo, rtol=1e-6, atol=1e-9)
    assert (flags.cpu().numpy() == 0).all()
