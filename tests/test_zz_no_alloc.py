"""spcn_normalize_noalloc (static per-GPU scratch) against spcn_normalize (caller workspace): the
same bytes and statistics, called through the C ABI twice in a row, the second call on a smaller
image, with and without a caller histogram (without one the histogram lives in the scratch)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def stats_tensors(dev, with_hist):
    st = {"p99_src": torch.empty(2, dtype=torch.float32, device=dev),
          "scale": torch.empty(2, dtype=torch.float32, device=dev),
          "flags": torch.empty(2, dtype=torch.int32, device=dev),
          "hist_hi": torch.empty(2, dtype=torch.float32, device=dev)}
    if with_hist:
        st["hist"] = torch.empty((2, 256), dtype=torch.uint64, device=dev)
    return st


def test_noalloc_equals_workspace_entry_point():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1901_03088_amd as S
    tgt = synth.make_image(1, 256, 256, device=DEV)
    wt = S.as_basis(tgt["W"], DEV)
    p = S.params()
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    # a large image first, then a smaller one (the scratch keeps the first call's contents), then a
    # range that overflows (the on-device retry reads and rewrites the scratch's range words)
    cases = [(0, 1024, 1536, p, True), (3, 300, 257, p, False), (5, 200, 300, S.params(hist_hi=(0.25, 0.25)), True)]
    for seed, h, w, pc, with_hist in cases:
        src = synth.make_image(seed, h, w, device=DEV)
        ws_ = S.as_basis(src["W"], DEV)
        ref, rst = S.spcn_normalize(src["img"], ws_, wt, sc, pc)
        out = torch.full_like(src["img"], 7)
        st = stats_tensors(DEV, with_hist)
        S.spcn_normalize_noalloc(src["img"], ws_, wt, sc, out, pc, stats=st)
        torch.cuda.synchronize()
        print(f"[noalloc] seed={seed} shape={h}x{w} hist={'caller' if with_hist else 'scratch'} "
              f"flags={st['flags'].tolist()} p99={st['p99_src'].tolist()}", flush=True)
        assert torch.equal(out, ref), (seed, h, w)
        for k in st:
            assert torch.equal(st[k].cpu(), rst[k].cpu()), (seed, k)
    # no statistics at all
    src = synth.make_image(8, 64, 96, device=DEV)
    ws_ = S.as_basis(src["W"], DEV)
    ref, _ = S.spcn_normalize(src["img"], ws_, wt, sc, p)
    out = torch.empty_like(src["img"])
    S.spcn_normalize_noalloc(src["img"], ws_, wt, sc, out, p)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy())
