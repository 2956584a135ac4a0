"""GPU parity of the batched persistent normalisation: every tile's output, percentile and scale
equal spcn_normalize on that tile alone (same kernels' arithmetic) and match the FP64 oracle on
the tile at the uint8 bar; plus the graph-captured batched pipeline (basis fit + normalise)."""
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


def make_batch(shapes, seed0=0):
    tiles = [synth.make_tile(seed0 + t, h, w, device=DEV) for t, (h, w) in enumerate(shapes)]
    srcs = [d["img"] for d in tiles]
    outs = [torch.empty_like(x) for x in srcs]
    return tiles, srcs, outs


def target(S, p):
    tgt = synth.target_image(256, device=DEV)
    wt = S.as_basis(tgt["W"], DEV)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    return tgt, wt, sc


@pytest.mark.parametrize("shapes", [
    [(256, 320), (64, 64), (1, 5), (300, 200), (512, 1024)],
    [(2048, 1984), (256, 256)] + [(64 * (1 + i % 5), 64 * (1 + (i * 7) % 9)) for i in range(40)],
])
def test_batched_equals_per_tile(S, orc, shapes):
    p = S.params()
    tiles, srcs, outs = make_batch(shapes)
    tgt, wt, sc = target(S, p)
    W = torch.stack([S.as_basis(d["W"], DEV) for d in tiles]).contiguous()
    table = S.tile_table(srcs, outs)
    total = sum(h * w for h, w in shapes)
    st = S.spcn_normalize_batched(table, len(shapes), total, W, wt, sc, p)
    torch.cuda.synchronize()
    flags = st["flags"].cpu().numpy(); p99 = st["p99"].cpu().numpy(); scale = st["scale"].cpu().numpy()
    scn = sc.cpu().numpy().astype(np.float64)
    for t, d in enumerate(tiles):
        ref, rst = S.spcn_normalize(srcs[t], W[t].contiguous(), wt, sc, p)
        torch.cuda.synchronize()
        assert torch.equal(ref, outs[t]), t
        assert np.array_equal(rst["p99_src"].cpu().numpy(), p99[t])
        assert np.array_equal(rst["flags"].cpu().numpy(), flags[t])
        if t < 6:
            o_out, o_st, o_hist = orc.normalize_u8(srcs[t].cpu().numpy(), orc.f32(orc.basis(d["W"])),
                                                   orc.f32(orc.basis(tgt["W"])), scn, lam=orc.f32(p.lambda_))
            dd = np.abs(o_out.astype(int) - outs[t].cpu().numpy().astype(int)).reshape(-1, 3).max(1)
            assert (dd <= 1).mean() >= 0.9999
            assert np.array_equal(o_st["P"].astype(np.float32), p99[t])


def test_batched_chunk_sizes_identical(S):
    """Every work-item size of the batched kernel gives the same bytes and statistics."""
    p = S.params()
    shapes = [(1024, 1024), (300, 200), (2048, 576), (64, 64), (1, 7)]
    tiles, srcs, outs = make_batch(shapes, seed0=50)
    tgt, wt, sc = target(S, p)
    W = torch.stack([S.as_basis(d["W"], DEV) for d in tiles]).contiguous()
    table = S.tile_table(srcs, outs)
    total = sum(h * w for h, w in shapes)
    saved = S.get_option(S.OPT_BATCH_CHUNK)
    ref = None
    try:
        for c in (12, 13, 14, 15, 16):
            S.set_option(S.OPT_BATCH_CHUNK, c)
            for o in outs:
                o.zero_()
            st = S.spcn_normalize_batched(table, len(shapes), total, W, wt, sc, p)
            torch.cuda.synchronize()
            cur = [o.cpu().numpy() for o in outs] + [st["p99"].cpu().numpy(), st["scale"].cpu().numpy(),
                                                     st["flags"].cpu().numpy()]
            if ref is None:
                ref = cur
            else:
                for a, b in zip(ref, cur):
                    assert np.array_equal(a, b), c
    finally:
        S.set_option(S.OPT_BATCH_CHUNK, saved)


def test_batched_bad_total_px_flags(S):
    p = S.params()
    tiles, srcs, outs = make_batch([(64, 64), (128, 64)])
    tgt, wt, sc = target(S, p)
    W = torch.stack([S.as_basis(d["W"], DEV) for d in tiles]).contiguous()
    table = S.tile_table(srcs, outs)
    # workspace sized for far fewer pixels than the tiles hold: nothing runs, every tile flagged
    st = S.spcn_normalize_batched(table, 2, 16, W, wt, sc, p)
    torch.cuda.synchronize()
    assert (st["flags"].cpu().numpy() & S.FLAG_BATCH).all()


def test_batched_pipeline_graph_replay(S, orc):
    """Batched basis fit + batched normalisation captured in one hipGraph and replayed several times
    with eager work in between; every replay equals the eager result."""
    p = S.params()
    shapes = [(256, 256), (320, 192), (128, 512), (64, 64)]
    tiles, srcs, outs = make_batch(shapes, seed0=10)
    tgt, wt, sc = target(S, p)
    table = S.tile_table(srcs, outs)
    total = sum(h * w for h, w in shapes)
    ws_b = S.workspace(S.workspace_size(S.OP_ESTIMATE_BATCHED, 0, len(shapes), 4096), DEV)
    ws_n = S.workspace(S.workspace_size(S.OP_NORMALIZE_BATCHED, total, len(shapes)), DEV)
    def run():
        W, _, _ = S.spcn_estimate_basis_batched(table, len(shapes), 4096, seed=7, p=p, want_p99=False, ws=ws_b)
        S.spcn_normalize_batched(table, len(shapes), total, W, wt, sc, p, ws=ws_n, stats=False)
        return W
    W0 = run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    W_eager = W0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Wg = run()
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for t in range(len(shapes)):
            assert torch.equal(eager[t], outs[t]), (rep, t)
        assert torch.equal(Wg, W_eager)
