"""GPU tests of the out-of-core normalisation of a slide in pinned host memory: the streamed result
equals spcn_normalize of the same image on the device byte for byte (one exact histogram over all
chunks), for several chunk sizes including single rows, ragged last chunks and one chunk, with
none, some or all chunks kept resident between the passes; it matches the FP64 oracle at the uint8
bar; and the copies wait for work still queued on the compute stream."""
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


def setup(S, seed, h, w):
    src = synth.make_image(seed, h, w, device=DEV)
    tgt = synth.make_image(1, 256, 256, device=DEV)
    p = S.params()
    ws, wt = S.as_basis(src["W"], DEV), S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    return src, tgt, p, ws, wt, sc


@pytest.mark.parametrize("h,w,chunk_rows", [(1024, 1024, 100), (777, 501, 64), (333, 257, 1000), (57, 33, 1),
                                            (512, 640, 512)])
def test_streamed_equals_device_normalize(S, orc, h, w, chunk_rows):
    src, tgt, p, ws, wt, sc = setup(S, 0, h, w)
    ref, st = S.spcn_normalize(src["img"], ws, wt, sc, p)
    host = src["img"].cpu().pin_memory()
    out, rst = S.spcn_normalize_streamed(host, ws, wt, sc, p, chunk_rows=chunk_rows)
    torch.cuda.synchronize()
    assert torch.equal(out, ref.cpu())
    assert torch.equal(rst["p99_src"], st["p99_src"]) and torch.equal(rst["flags"], st["flags"])
    if h * w <= 1 << 20:
        o_out, o_st, _ = orc.normalize_u8(host.numpy(), orc.f32(orc.basis(src["W"])), orc.f32(orc.basis(tgt["W"])),
                                          sc.cpu().numpy().astype(np.float64), lam=orc.f32(p.lambda_))
        dd = np.abs(o_out.astype(int) - out.numpy().astype(int)).reshape(-1, 3).max(1)
        assert (dd <= 1).mean() >= 0.9999


def test_streamed_repeat_and_separate_copy_streams(S):
    """Two calls in a row (events reused) with distinct in/out copy streams."""
    src, tgt, p, ws, wt, sc = setup(S, 3, 600, 400)
    ref, _ = S.spcn_normalize(src["img"], ws, wt, sc, p)
    host = src["img"].cpu().pin_memory()
    cin, cout = torch.cuda.Stream(), torch.cuda.Stream()
    for rows in (50, 77):
        out, _ = S.spcn_normalize_streamed(host, ws, wt, sc, p, chunk_rows=rows, copy_in=cin, copy_out=cout)
        torch.cuda.synchronize()
        assert torch.equal(out, ref.cpu())


@pytest.mark.parametrize("resident", [1, 3, 100])
def test_streamed_resident_chunks(S, resident):
    """A larger workspace keeps the first chunks on the device between the passes (recoloured in
    place): same bytes as the in-HBM path, whatever the number kept (all of them included)."""
    h, w, rows = 777, 501, 64
    src, tgt, p, ws, wt, sc = setup(S, 5, h, w)
    ref, st = S.spcn_normalize(src["img"], ws, wt, sc, p)
    host = src["img"].cpu().pin_memory()
    base = S.workspace_size(S.OP_STREAM_NORMALIZE, w, rows, 0)
    chunk = (3 * rows * w + 255) // 256 * 256
    n_chunks = (h + rows - 1) // rows
    wsb = S.workspace(base + resident * chunk, DEV)
    assert S.stream_resident_chunks(h, w, rows, base + resident * chunk) == min(resident, n_chunks)
    out, rst = S.spcn_normalize_streamed(host, ws, wt, sc, p, chunk_rows=rows, ws=wsb)
    torch.cuda.synchronize()
    assert torch.equal(out, ref.cpu())
    assert torch.equal(rst["p99_src"], st["p99_src"]) and torch.equal(rst["scale"], st["scale"])


def test_streamed_waits_for_queued_compute_work(S):
    """The host input is written by a copy still queued on the compute stream when the streamed call
    is made (no synchronisation in between): the call's copies must wait for it."""
    src, tgt, p, ws, wt, sc = setup(S, 6, 640, 480)
    ref, _ = S.spcn_normalize(src["img"], ws, wt, sc, p)
    torch.cuda.synchronize()
    host = torch.zeros((640, 480, 3), dtype=torch.uint8).pin_memory()
    busy = torch.empty((4096, 4096), device=DEV)
    busy.normal_()
    for _ in range(20):          # keep the compute stream busy for a while
        busy = busy @ busy.T * 1e-3
    host.copy_(src["img"], non_blocking=True)   # device -> pinned host, queued behind the products
    out, _ = S.spcn_normalize_streamed(host, ws, wt, sc, p, chunk_rows=100)
    torch.cuda.synchronize()
    assert torch.equal(out, ref.cpu())
