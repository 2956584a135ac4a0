"""GPU parity of the differentiable float path with the FP64 oracle: forward outputs, the exact
order statistic (value, and validity of the selected index), and the adjoint (input, target-basis
and scale gradients), the latter compared with the oracle's analytic adjoint, which the CPU tests
pin to FP64 finite differences.  The loss is L = sum(w * y^2) with fixed random weights w, so the
incoming gradient is 2 w y.

Tolerances: outputs 2e-5 absolute (values in [0, 1]); percentile 1e-5 relative; input gradients
per element |g - g_ref| <= 1e-3 |g_ref| + 1e-5 max|g_ref| (the absolute floor covers elements whose
FP32 terms cancel; the sum over a pixel's channels runs over terms of the sample's gradient scale);
the selected order-statistic pixels within 1e-3 relative on every channel; target-basis and scale
gradients 1e-3 relative.  The only pixels excused are those the oracle marks as within 1e-4 of an
active-set change of Eq. (2), where FP32 and FP64 may legitimately solve on different faces."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
RTOL_G, FLOOR_G, MARGIN = 1e-3, 1e-5, 1e-4


@pytest.fixture(scope="module")
def S():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_1901_03088_amd as s
    return s


def batch(n, size, seed=40):
    x, Ws, Wt, wts = synth.float_batch(n, size, seed, device=DEV)
    return x.contiguous(), Ws, Wt, wts


def per_sample(S, Ws):
    return torch.stack([S.as_basis(W, DEV) for W in Ws]).contiguous()


def check_forward(orc, i, xs, yg, Pg, selg, Ws, Wt, sci, lam):
    Wsi, Wti = orc.f32(orc.basis(Ws)), orc.f32(orc.basis(Wt))
    yo, Po, isto, Ho, flo = orc.forward_f32(xs, Wsi, Wti, sci, lam=orc.f32(lam))
    assert np.abs(yg - yo).max() < 2e-5, (i, np.abs(yg - yo).max())
    assert np.allclose(Pg, Po, rtol=1e-5), (i, Pg, Po)
    for j in range(2):
        if Po[j] > 0:   # the GPU's pixel holds (in FP64) the oracle's order statistic up to FP32 error
            assert abs(Ho[j, selg[j]] - Po[j]) <= 2e-5 * Po[j], (i, j)
    return Wsi, Wti, Po


def check_backward(orc, i, xs, gy, gxg, gwg, gsg, Wsi, Wti, sci, selg, Po, lam):
    gxo, gwo, gso, _ = orc.backward_f32(xs, Wsi, Wti, sci, gy, lam=orc.f32(lam), istar=selg)
    n_px = xs.shape[1] * xs.shape[2]
    g_o, g_g = gxo.reshape(3, n_px), gxg.reshape(3, n_px)
    err = np.abs(g_g - g_o)
    bad = err > RTOL_G * np.abs(g_o) + FLOOR_G * np.abs(g_o).max()
    near = orc.active_margin_f32(xs, Wsi, lam=orc.f32(lam)) < MARGIN
    bad_px = bad.any(0)
    print(f"[f32 {i}] max|dgrad|/max|g| {err.max() / np.abs(g_o).max():.2e}; off-tolerance px {int(bad_px.sum())} "
          f"(near an active-set change: {int((bad_px & near).sum())} of {int(near.sum())} such px)", flush=True)
    assert not (bad_px & ~near).any(), (i, np.nonzero(bad_px & ~near)[0][:10])
    # the order-statistic term lands on the selected pixels: compare them explicitly
    for j in range(2):
        if Po[j] > 0:
            k = int(selg[j])
            assert np.allclose(g_g[:, k], g_o[:, k], rtol=RTOL_G, atol=FLOOR_G * np.abs(g_o).max()), (i, j, k)
    assert np.allclose(gwg, gwo, rtol=RTOL_G, atol=1e-6 * np.abs(gwo).max()), (i, gwg, gwo)
    assert np.allclose(gsg, gso, rtol=RTOL_G, atol=1e-6 * np.abs(gso).max()), (i, gsg, gso)


def run_case(S, orc, n, size, scale_shared=True, lam=0.01):
    x, Ws, Wt, wts = batch(n, size)
    p = S.float_params(lam=lam)
    ws, wt = per_sample(S, Ws), per_sample(S, Wt)
    sc = torch.tensor([0.9, 1.1], dtype=torch.float32, device=DEV) if scale_shared else \
        torch.rand((n, 2), device=DEV) * 0.5 + 0.75
    y, saved = S.spcn_normalize_f32(x, ws, wt, sc, p)
    gy = 2.0 * wts * y
    # per-sample gradients (a shared scale given once per sample: same forward, gradients not summed)
    gx, gw, gs = S.spcn_normalize_backward(x, ws, wt, sc.expand(n, 2).contiguous(), saved, gy, p)
    torch.cuda.synchronize()
    xs_all = x.cpu().numpy().astype(np.float64)
    for i in range(n):
        sci = sc.cpu().numpy().astype(np.float64) if scale_shared else sc[i].cpu().numpy().astype(np.float64)
        selg = saved["sel"][i].cpu().numpy()
        Wsi, Wti, Po = check_forward(orc, i, xs_all[i], y[i].cpu().numpy(), saved["p99"][i].cpu().numpy(), selg,
                                     Ws[i], Wt[i], sci, lam)
        check_backward(orc, i, xs_all[i], gy[i].cpu().numpy().astype(np.float64), gx[i].cpu().numpy(),
                       gw[i].cpu().numpy(), gs[i].cpu().numpy(), Wsi, Wti, sci, selg, Po, lam)


def test_f32_small(S, orc):
    run_case(S, orc, 3, 64)


def test_f32_ragged_and_lambda0(S, orc):
    run_case(S, orc, 2, 37, lam=0.0, scale_shared=False)


def test_f32_config4_shape(S, orc):
    """64 x 3 x 512 x 512 forward + backward at the benchmark shape: every sample's output,
    percentile and selected pixels against the oracle; the full adjoint on 4 seeded samples."""
    n, size = 64, 512
    x, Ws, Wt, wts = batch(n, size)
    p = S.float_params()
    ws, wt = per_sample(S, Ws), per_sample(S, Wt)
    sc = torch.tensor([0.9, 1.1], dtype=torch.float32, device=DEV)
    y, saved = S.spcn_normalize_f32(x, ws, wt, sc, p)
    gy = 2.0 * wts * y
    gx, gw, gs = S.spcn_normalize_backward(x, ws, wt, sc.expand(n, 2).contiguous(), saved, gy, p)
    torch.cuda.synchronize()
    sci = sc.cpu().numpy().astype(np.float64)
    grad_samples = set(np.random.default_rng(4).choice(n, 4, replace=False).tolist())
    for i in range(n):
        xs = x[i].cpu().numpy().astype(np.float64)
        selg = saved["sel"][i].cpu().numpy()
        Wsi, Wti, Po = check_forward(orc, i, xs, y[i].cpu().numpy(), saved["p99"][i].cpu().numpy(), selg,
                                     Ws[i], Wt[i], sci, 0.01)
        if i in grad_samples:
            check_backward(orc, i, xs, gy[i].cpu().numpy().astype(np.float64), gx[i].cpu().numpy(),
                           gw[i].cpu().numpy(), gs[i].cpu().numpy(), Wsi, Wti, sci, selg, Po, 0.01)


def test_autograd_function(S):
    x, Ws, Wt, wts = batch(2, 48)
    p = S.float_params()
    ws = per_sample(S, Ws)
    wt = S.as_basis(Wt[0], DEV).requires_grad_(True)
    sc = torch.tensor([0.9, 1.1], dtype=torch.float32, device=DEV, requires_grad=True)
    xr = x.clone().requires_grad_(True)
    y = S.SPCNNormalize.apply(xr, ws, wt, sc, p)
    (wts * y * y).sum().backward()
    torch.cuda.synchronize()
    y2, saved = S.spcn_normalize_f32(x, ws, wt.detach(), sc.detach(), p)
    gx, gw, gs = S.spcn_normalize_backward(x, ws, wt.detach(), sc.detach(), saved, 2.0 * wts * y2, p)
    assert gw.shape == (6,) and gs.shape == (2,)      # shared parameters: summed by the library
    assert torch.equal(xr.grad, gx) and torch.equal(wt.grad, gw) and torch.equal(sc.grad, gs)
    # the same parameters given per sample: per-sample gradients whose sum is the shared one
    n = x.shape[0]
    wt_n, sc_n = wt.detach().expand(n, 6).contiguous(), sc.detach().expand(n, 2).contiguous()
    gx_n, gw_n, gs_n = S.spcn_normalize_backward(x, ws, wt_n, sc_n, saved, 2.0 * wts * y2, p)
    assert gw_n.shape == (n, 6) and gs_n.shape == (n, 2)
    assert torch.equal(gx_n, gx)
    assert torch.allclose(gw, gw_n.double().sum(0).float(), rtol=1e-6, atol=1e-7 * float(gw_n.abs().max()))
    assert torch.allclose(gs, gs_n.double().sum(0).float(), rtol=1e-6, atol=1e-7 * float(gs_n.abs().max()))
