#!/usr/bin/env python3
"""Benchmark of the SPCN hot path on one MI355X: a 50000 x 40000 (2 Gpixel) synthetic slide,
~60% background, normalised to one target.

One step = the whole path for the slide: basis estimation from 200k sampled tissue pixels (sparse
NMF, 50 rounds, the samples' percentile and the histogram range derived from it) + pass 1 (densities
+ exact histogram, with the device-side range check and its gated repeat) + pass 2 (percentile,
recolour, uint8 write).  The flags of the timed step are checked: no overflow, timeout or skip.
Inputs are resident in HBM before the timed region.  Extras (same JSON line): the batched workload
(512 tiles in one graph) against a per-tile loop, and forward+backward of the float path against
forward only, and the FP32 densities of an 8192^2 image.  Prints ONE JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload slide|cfg1|small]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Mpixel/s SPCN normalize at 2 Gpx + % HBM peak; batched & fwd+bwd Mpx/s"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def build_slide(workload: str, dev):
    import torch
    import synth
    if workload == "slide":
        img, W, plan = synth.make_slide(device=dev)
        desc = {"workload": "gigapixel_slide", "height": synth.SLIDE_H, "width": synth.SLIDE_W,
                "block": synth.SLIDE_BLOCK, "tissue_slots": sum(1 for s in plan if s[4]), "slots": len(plan)}
    elif workload == "cfg1":
        d = synth.config1(device=dev)
        img, W = d["img"], d["W"]
        desc = {"workload": "single_image_8192", "height": 8192, "width": 8192}
    else:
        d = synth.make_image(0, 1024, 1024, device=dev)
        img, W = d["img"], d["W"]
        desc = {"workload": "small_1024", "height": 1024, "width": 1024}
    torch.cuda.synchronize()
    return img, W, desc


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(img_dev, W_src, W_tgt, scale_tgt, n_px_total: int, hist_hi=(8.0, 8.0), n_samples: int = 200000,
                 bands: int = 8, band_rows: int = 1000, single_rows: int = 100):
    """The FP64 oracle, as it stands, timed stage by stage on the host cores: pass 1 (densities of
    every pixel + the non-white histogram) and pass 2 (densities again + recolour + rounding) on
    `bands` bands of `band_rows` rows spread over the slide, the percentile from their histogram,
    and the sparse NMF on n_samples sampled tissue pixels of those bands (50 rounds).  The value is
    the rate of the whole step at the slide's size: n_px_total / (pass-1 and pass-2 time per pixel
    x n_px_total + percentile + NMF).  The two passes are timed again on one thread (a smaller band)."""
    import ctypes
    import numpy as np
    import oracle as orc
    H_img, W_img = int(img_dev.shape[0]), int(img_dev.shape[1])
    starts = [int(k * (H_img - band_rows) / max(1, bands - 1)) for k in range(bands)]
    sample = np.concatenate([img_dev[r0:r0 + band_rows].cpu().numpy() for r0 in starts])
    Ws, Wt = orc.f32(orc.basis(W_src)), orc.f32(orc.basis(W_tgt))
    sc = np.asarray(scale_tgt, dtype=np.float64)
    lam = orc.f32(0.01)

    def passes(img):
        t0 = time.perf_counter()
        H, m = orc.densities_u8(img, Ws, lam=lam)
        hist = orc.histogram(H, m, hist_hi, 256)
        t1 = time.perf_counter()
        P = [orc.percentile_hist(hist[j], hist_hi[j], orc.q_of(99.0))[0] for j in range(2)]
        t2 = time.perf_counter()
        del H, m
        orc.recolor_u8(img, Ws, Wt, sc, np.array(P), lam=lam)
        t3 = time.perf_counter()
        return t1 - t0, t2 - t1, t3 - t2, P

    n = sample.shape[0] * sample.shape[1]
    t_p1, t_fin, t_p2, _ = passes(sample)
    idx = orc.sample_tissue(sample, n_samples, 2024, 660)
    V = orc.od_samples(sample, idx)
    H0 = np.array([0.65, 0.70, 0.29]); E0 = np.array([0.07, 0.99, 0.11])
    W_init = orc.f32(np.stack([H0 / np.linalg.norm(H0), E0 / np.linalg.norm(E0)], axis=1))
    t0 = time.perf_counter()
    orc.nmf(V, orc.f32(0.1), 50, W_init, 99.0)
    t_nmf = time.perf_counter() - t0
    gomp = None
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    try:   # the same passes on one thread (the oracle's loops are OpenMP loops)
        gomp = ctypes.CDLL("libgomp.so.1")
        threads = gomp.omp_get_max_threads()
        gomp.omp_set_num_threads(1)
        one = sample[:single_rows]
        s1, _, s2, _ = passes(one)
        n1 = one.shape[0] * one.shape[1]
        single = {"pixels": n1, "pass1_Mpx_s": round(n1 / s1 / 1e6, 2), "pass2_Mpx_s": round(n1 / s2 / 1e6, 2)}
    except OSError:
        single = None
    finally:
        if gomp is not None:
            gomp.omp_set_num_threads(threads)
    per_px = (t_p1 + t_p2) / n
    step_s = per_px * n_px_total + t_fin + t_nmf
    return {"value": round(n_px_total / step_s / 1e6, 1), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": f"{bands} bands of {band_rows} rows x {W_img} px ({n / 1e6:.0f} Mpixel) spread over the slide "
                      f"for the two passes, {n_samples} tissue samples of them for the NMF; step time scaled to "
                      f"{n_px_total / 1e9:.1f} Gpixel: {step_s:.1f} s",
            "stages": {"pass1_Mpx_s": round(n / t_p1 / 1e6, 1), "percentile_ms": round(t_fin * 1e3, 3),
                       "pass2_Mpx_s": round(n / t_p2 / 1e6, 1), "nmf_s": round(t_nmf, 3),
                       "nmf_samples": int(V.shape[1]), "nmf_rounds": 50,
                       "normalize_Mpx_s": round(1.0 / per_px / 1e6, 1)},
            "single_thread": single}


P1_KERNELS = ["k_pass1<1, 64, 4, 4>", "k_pass1<2, 64, 4, 4>", "k_pass1<4, 32, 4, 4>", "k_pass1<8, 16, 4, 4>",
              "k_pass1<1, 32, 2, 8>", "k_pass1<2, 16, 2, 8>", "k_pass1g<true, 1024, 4, 4>",
              "k_pass1g<true, 1024, 2, 4>", "k_pass1g<false, 768, 2, 6>", "k_pass1g<false, 512, 2, 4>"]
P2_KERNELS = ["k_pass2<1, 256>", "k_pass2<4, 256>", "k_pass2<16, 1024>", "k_pass2g<1, 256>", "k_pass2g<1, 512>",
              "k_pass2g<16, 1024>"]
TRAFFIC_SOURCES = ["paper_1901_03088_amd/csrc/spcn_passes.hpp", "paper_1901_03088_amd/csrc/spcn_u8.hip",
                   "paper_1901_03088_amd/csrc/spcn_device.hpp", "paper_1901_03088_amd/csrc/spcn_internal.h"]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary (rocprofv3 FETCH_SIZE /
    WRITE_SIZE, calibrated), or None if the summary is for other sources, another workload or
    lacks this kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if workload != "gigapixel_slide" or not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get("kernels", {}).get(kernel)
    if not rec or rec.get("write_bytes") is None:
        return None
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sources_sha256"):
        return None
    return round(rec["read_bytes"] + rec["write_bytes"])


def timed(fn, steps, warmup, stream):
    """Mean ms of fn() over `steps` runs bracketed by events on `stream` (after `warmup` runs)."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))


def bench_batched(dev, S, synth, steps, warmup, n_tiles=512, loop=True, tune=True):
    """512 uneven tiles (sides 256..2048 step 64), per-tile basis fit (4096 samples, 50 rounds,
    lambda 0.1) and normalisation to one target, captured in one hipGraph and replayed; against a
    per-tile loop of the plain single-image path (same work, same results) unless loop is False."""
    import torch
    shapes = synth.tile_shapes(n_tiles)
    srcs = [synth.make_tile(t, h, w, device=dev)["img"] for t, (h, w) in enumerate(shapes)]
    outs = [torch.empty_like(x) for x in srcs]
    total = sum(h * w for h, w in shapes)
    table = S.tile_table(srcs, outs)
    p = S.params()
    tgt = synth.target_image(device=dev)
    wt = S.as_basis(tgt["W"], dev)
    _, _, sc, _ = S.spcn_densities(tgt["img"], wt, p, want_h=False)
    ws_b = S.workspace(S.workspace_size(S.OP_ESTIMATE_BATCHED, 0, n_tiles, 4096), dev)
    ws_n = S.workspace(S.workspace_size(S.OP_NORMALIZE_BATCHED, total, n_tiles), dev)
    hh_t = torch.empty((n_tiles, 2), dtype=torch.float32, device=dev)   # per-tile ranges from the fits
    p_t = S.params(hist_hi_dev=hh_t)

    def run():
        W, _, _ = S.spcn_estimate_basis_batched(table, n_tiles, 4096, seed=30000, p=p, want_p99=False, ws=ws_b,
                                                hist_hi_out=hh_t)
        S.spcn_normalize_batched(table, n_tiles, total, W, wt, sc, p_t, ws=ws_n, stats=False)
        return W
    from paper_1901_03088_amd import autotune
    W_fit = run()
    tuned = (autotune.tune_batched(table, n_tiles, total, W_fit, wt, sc, outs, p_t) if tune else
             {"options": {"batch_chunk_log2": S.get_option(S.OPT_BATCH_CHUNK)}})
    run()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    stream = torch.cuda.current_stream()
    ms_graph = timed(g.replay, steps, warmup, stream)
    res = {"tiles": n_tiles, "pixels": total, "autotune": tuned["options"], "graph_ms": round(ms_graph, 3),
           "graph_Mpx_s": round(total / ms_graph / 1e3, 1)}
    if not loop:
        return res
    # the same work tile by tile through the single-image entry points (same fits, same ranges, no
    # automatic retry, so the same bytes), eagerly and captured into one graph
    ws1 = S.workspace(S.workspace_size(S.OP_ESTIMATE_BASIS, 0, 1, 4096), dev)
    wsn1 = S.workspace(S.workspace_size(S.OP_NORMALIZE), dev)
    w1 = torch.empty((n_tiles, 6), dtype=torch.float32, device=dev)
    hh1 = torch.empty((n_tiles, 2), dtype=torch.float32, device=dev)
    p1 = [S.params(hist_hi_dev=hh1[t]) for t in range(n_tiles)]

    def per_tile():
        for t in range(n_tiles):
            S.spcn_estimate_basis(srcs[t], 4096, seed=30000 + t, p=p, lambda_nmf=0.1, n_iter=50, want_p99=False,
                                  w_out=w1[t], ws=ws1, hist_hi_out=hh1[t])
            S.spcn_normalize(srcs[t], w1[t], wt, sc, p1[t], out=outs[t], stats=False, ws=wsn1)
    ms_loop = timed(per_tile, max(1, steps // 4), 1, stream)
    per_tile()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        per_tile()
    torch.cuda.current_stream().wait_stream(side)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        per_tile()
    ms_loop_graph = timed(g2.replay, max(2, steps // 2), 1, stream)
    del g2
    return dict(res, per_tile_loop_ms=round(ms_loop, 3), per_tile_loop_Mpx_s=round(total / ms_loop / 1e3, 1),
                per_tile_graph_ms=round(ms_loop_graph, 3),
                per_tile_graph_Mpx_s=round(total / ms_loop_graph / 1e3, 1),
                speedup_vs_eager_loop=round(ms_loop / ms_graph, 2),
                speedup_vs_graph_loop=round(ms_loop_graph / ms_graph, 2))


def bench_densities(dev, S, synth, steps, warmup, size=8192):
    """spcn_densities with the FP32 density planes on the 8192 x 8192 single image (67 Mpixel): the
    whole call (set-up, pass 1 writing the densities, range check, gated repeat, percentile).  The
    algorithmic traffic is 3 B/px read + 8 B/px written."""
    import torch
    d = synth.config1(size, device=dev)
    img, w = d["img"], S.as_basis(d["W"], dev)
    n = size * size
    p = S.params()
    h = torch.empty((2, n), dtype=torch.float32, device=dev)
    hist = torch.empty((2, 256), dtype=torch.uint64, device=dev)
    p99 = torch.empty(2, dtype=torch.float32, device=dev)
    flags = torch.empty(2, dtype=torch.int32, device=dev)
    ws = S.workspace(S.workspace_size(S.OP_DENSITIES), dev)
    stream = torch.cuda.current_stream()
    ms = timed(lambda: S.spcn_densities(img, w, p, h_out=h, hist_out=hist, p99_out=p99, flags_out=flags, ws=ws),
               steps, warmup, stream)
    gbs = 11.0 * n / (ms / 1e3) / 1e9
    return {"workload": "single_image_8192", "pixels": n, "ms": round(ms, 4), "Mpx_s": round(n / ms / 1e3, 1),
            "bytes_per_px": 11, "GBs": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
            "flags": [int(v) for v in flags.cpu()]}


def bench_fwdbwd(dev, S, synth, steps, warmup, n=64, size=512):
    """Differentiable path: 64 x 3 x 512 x 512 float images, per-sample target bases, forward +
    backward of L = sum(w * y^2) (fixed random weights w, so dL/dy = 2 w y, one elementwise product
    timed with the step), against forward only."""
    import torch
    x, Ws, Wt, wts = synth.float_batch(n, size, device=dev)
    p = S.float_params()
    ws = torch.stack([S.as_basis(W, dev) for W in Ws]).contiguous()
    wt = torch.stack([S.as_basis(W, dev) for W in Wt]).contiguous()
    sc = torch.tensor([0.9, 1.1], dtype=torch.float32, device=dev)
    fws = S.workspace(S.workspace_size(S.OP_FORWARD_F32, size * size, n), dev)
    bws = S.workspace(S.workspace_size(S.OP_BACKWARD_F32, size * size, n), dev)
    y = torch.empty_like(x)
    gy = torch.empty_like(x)
    w2 = 2.0 * wts
    stream = torch.cuda.current_stream()
    state = {}

    def fwd():
        state["saved"] = S.spcn_normalize_f32(x, ws, wt, sc, p, y=y, ws=fws)[1]

    def fwd_bwd():
        fwd()
        torch.mul(w2, y, out=gy)                    # dL/dy of L = sum(w * y^2)
        S.spcn_normalize_backward(x, ws, wt, sc, state["saved"], gy, p, ws=bws)
    ms_f = timed(fwd, steps, warmup, stream)
    ms_fb = timed(fwd_bwd, steps, warmup, stream)
    ms_loss = timed(lambda: torch.mul(w2, y, out=gy), steps, warmup, stream)
    px = n * size * size
    return {"batch": [n, 3, size, size], "loss": "sum(w * y^2)", "forward_ms": round(ms_f, 3),
            "forward_Mpx_s": round(px / ms_f / 1e3, 1), "fwd_bwd_ms": round(ms_fb, 3),
            "fwd_bwd_Mpx_s": round(px / ms_fb / 1e3, 1), "loss_grad_ms": round(ms_loss, 3),
            "forward_bytes_per_px": 48, "backward_bytes_per_px": 36}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slide", choices=["slide", "cfg1", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the batched and forward+backward measurements")
    ap.add_argument("--only", choices=["batched", "fwdbwd", "densities"], default=None,
                    help="run one extra workload alone (the batched graph without the per-tile loop, the "
                         "differentiable batch, or the 8192^2 densities), for profiling; no slide step")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library's default kernel variants (for profiling runs, whose traces should "
                         "hold only the timed kernels)")
    ap.add_argument("--ceilings", action="store_true",
                    help="also time the bandwidth reference kernels on the slide's buffers: a copy of the slide "
                         "into the output buffer and a read-only pass over the slide")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB read + 1 GiB write elementwise kernel (torch.neg on float32), "
                         "whose FETCH_SIZE / WRITE_SIZE counters calibrate the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md for how the "
              "histogram would be all-reduced across shards); run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1901_03088_amd as S
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        if args.only == "batched":
            r = bench_batched(dev, S, synth, args.steps, args.warmup, loop=False, tune=args.autotune)
        elif args.only == "densities":
            r = bench_densities(dev, S, synth, args.steps, args.warmup)
        else:
            r = bench_fwdbwd(dev, S, synth, args.steps, args.warmup)
        log(f"[bench] {args.only} {r}")
        print(json.dumps(dict(only=args.only, steps=args.steps, warmup=args.warmup, **r)))
        return 0
    t0 = time.time()
    img, W_src, desc = build_slide(args.workload, dev)
    Hh, Ww = int(img.shape[0]), int(img.shape[1])
    n_px = Hh * Ww
    log(f"[bench] input {desc} built in {time.time() - t0:.1f} s ({n_px / 1e9:.2f} Gpixel)")
    tgt = synth.target_image(device=dev)
    p = S.params()
    w_src = S.as_basis(W_src, dev)
    w_tgt = S.as_basis(tgt["W"], dev)
    _, _, scale_tgt, _ = S.spcn_densities(tgt["img"], w_tgt, p, want_h=False)
    out = torch.empty_like(img)
    hist = torch.empty((2, 256), dtype=torch.uint64, device=dev)
    w_fit = torch.empty(6, dtype=torch.float32, device=dev)
    hh_fit = torch.empty(2, dtype=torch.float32, device=dev)     # range from the basis sample
    hh_used = torch.empty(2, dtype=torch.float32, device=dev)    # range the histogram was built over
    p_fit = S.params(hist_hi_dev=hh_fit)
    p_used = S.params(hist_hi_dev=hh_used)
    n_samples = 200000
    ws_fit = S.workspace(S.workspace_size(S.OP_ESTIMATE_BASIS, n_px, 1, n_samples), dev)
    ws_d = S.workspace(S.workspace_size(S.OP_DENSITIES), dev)
    st = {"p99_src": torch.empty(2, dtype=torch.float32, device=dev),
          "scale": torch.empty(2, dtype=torch.float32, device=dev),
          "flags": torch.empty(2, dtype=torch.int32, device=dev),
          "hist_hi": torch.empty(2, dtype=torch.float32, device=dev)}
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    from paper_1901_03088_amd import autotune
    # tune on the basis the step fits (the bin distribution, hence LDS contention, depends on it)
    S.spcn_estimate_basis(img, n_samples, seed=2024, p=S.params(), lambda_nmf=0.1, n_iter=50, want_p99=False,
                          w_out=w_fit, ws=ws_fit, hist_hi_out=hh_fit)
    tuned = (autotune.tune_image(img, w_fit, w_tgt, scale_tgt, p_fit) if args.autotune else
             {"options": {"p1_variant": S.get_option(S.OPT_P1_VARIANT), "p2_variant": S.get_option(S.OPT_P2_VARIANT),
                          "p2_blocks_per_cu": S.get_option(S.OPT_P2_BLOCKS_PER_CU)}})
    log(f"[bench] autotune chose {tuned['options']}")

    def step(ev=None):
        # one step = the whole path for the slide: basis fit (200k samples, sample percentile and
        # range) -> pass 1 (range check, gated repeat) -> pass 2
        if ev is not None:
            ev[0].record(stream)
        S.spcn_estimate_basis(img, n_samples, seed=2024, p=S.params(), lambda_nmf=0.1, n_iter=50, want_p99=False,
                              w_out=w_fit, ws=ws_fit, hist_hi_out=hh_fit)
        if ev is not None:
            ev[1].record(stream)
        S.spcn_densities(img, w_fit, p_fit, want_h=False, hist_out=hist, finalize=False, hist_hi_out=hh_used,
                         ws=ws_d)
        if ev is not None:
            ev[2].record(stream)
        S.spcn_recolor(img, w_fit, w_tgt, scale_tgt, hist, p_used, out=out, stats=st)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    pb = [e[0].elapsed_time(e[1]) for e in evs]
    p1 = [e[1].elapsed_time(e[2]) for e in evs]
    p2 = [e[2].elapsed_time(e[3]) for e in evs]
    tot = [e[0].elapsed_time(e[3]) for e in evs]
    ms_step = float(np.mean(tot))
    value = n_px / (ms_step / 1e3) / 1e6
    pbm, p1m, p2m = float(np.mean(pb)), float(np.mean(p1)), float(np.mean(p2))
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (wall {wall * 1e3 / args.steps:.3f}), "
        f"basis {pbm:.3f} ms, pass1 {p1m:.3f} ms, pass2 {p2m:.3f} ms")
    step_flags = [int(v) for v in st["flags"].cpu()]
    bad = S.FLAG_RANGE | S.FLAG_TIMEOUT | S.FLAG_BATCH | S.FLAG_NO_TISSUE | S.FLAG_BASIS
    if any(f & bad for f in step_flags):
        log(f"[bench] the timed step raised flags {step_flags}")
        return 3

    # roofline of the dominant kernel (algorithmic bytes: 3 B/px read in pass 1; 3 read + 3 written in pass 2)
    k1 = P1_KERNELS[S.get_option(S.OPT_P1_VARIANT)]
    k2 = P2_KERNELS[S.get_option(S.OPT_P2_VARIANT)]
    k_name, k_ms, k_bytes = (k2, p2m, 6.0 * n_px) if p2m >= p1m else (k1, p1m, 3.0 * n_px)
    achieved = k_bytes / (k_ms / 1e3) / 1e9
    norm_ms = p1m + p2m
    path_gbs = 9.0 * n_px / (norm_ms / 1e3) / 1e9
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(desc, pixels=n_px, background_frac=0.6, lambda_density=0.01, io="uint8 RGB HWC"),
        "roofline": {"bound": "hbm", "kernel": k_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(k_name, desc["workload"]),
                     "algorithmic_bytes": round(k_bytes)},
        "autotune": tuned["options"],
        "path": {"flags": step_flags, "hist_hi": [float(v) for v in st["hist_hi"].cpu()],
                 "p99_src": [float(v) for v in st["p99_src"].cpu()],
                 "basis_fit_ms": round(pbm, 4), "pass1_ms": round(p1m, 4), "pass2_ms": round(p2m, 4),
                 "normalize_ms": round(norm_ms, 4), "normalize_Mpx_s": round(n_px / norm_ms / 1e3, 1),
                 "normalize_GBs_9B_per_px": round(path_gbs, 1),
                 "normalize_frac_of_peak": round(path_gbs / HBM_PEAK_GBS, 4)},
    }
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).uniform_()
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        res["copy_calibration"] = {"kernel": "torch.neg float32", "read_bytes": a.numel() * 4,
                                   "write_bytes": b.numel() * 4, "launches": 3}
        del a, b
    if args.ceilings:
        # what plain library kernels reach on the slide's own buffers: a copy of the input into the
        # output (6 GB read + 6 GB written, pass 2's traffic) and a read-only reduction of the input
        # (6 GB read, pass 1's traffic)
        # (streaming cache policy as the passes use, and the default policy)
        ws_probe = S.workspace(S.workspace_size(S.OP_BANDWIDTH_PROBE), dev)
        ms = {}
        for mode in range(4):
            dst = out if mode in (0, 2) else None
            ms[mode] = timed(lambda: S.spcn_bandwidth_probe(img, dst, mode, ws=ws_probe), args.steps, args.warmup,
                             stream)
        ms_tcopy = timed(lambda: out.copy_(img), args.steps, args.warmup, stream)
        def ceil(mode, what, per_px):
            return {"kernel": f"k_probe {what} (spcn_bandwidth_probe mode {mode})", "ms": round(ms[mode], 4),
                    "GBs": round(per_px * n_px / (ms[mode] / 1e3) / 1e9, 1)}
        res["ceilings"] = {
            "copy": ceil(0, "copy, streaming policy", 6.0), "read": ceil(1, "read, streaming policy", 3.0),
            "copy_default_policy": ceil(2, "copy, default policy", 6.0),
            "read_default_policy": ceil(3, "read, default policy", 3.0),
            "torch_copy": {"kernel": "torch copy_ uint8", "ms": round(ms_tcopy, 4),
                           "GBs": round(6.0 * n_px / (ms_tcopy / 1e3) / 1e9, 1)}}
        log(f"[bench] ceilings {res['ceilings']}")
    if not args.no_cpu_baseline:
        t_cpu = time.time()
        res["cpu_baseline"] = cpu_baseline(img, W_src, tgt["W"], scale_tgt.cpu().numpy(), n_px,
                                           hist_hi=[float(v) for v in st["hist_hi"].cpu()])
        log(f"[bench] cpu baseline {res['cpu_baseline']} ({time.time() - t_cpu:.0f} s)")
    if args.extras:
        # channel-wise background intensity (Sec. 3.1 item 1): 100k background samples of the slide
        i0_dev = torch.empty(3, dtype=torch.float32, device=dev)
        ws_i0 = S.workspace(S.workspace_size(S.OP_ESTIMATE_I0, 0, 0, 100000), dev)
        ms_i0 = timed(lambda: S.spcn_estimate_i0(img, 100000, seed=7, i0_out=i0_dev, ws=ws_i0), args.steps,
                      args.warmup, stream)
        res.setdefault("extras", {})["i0_estimate"] = {"samples": 100000, "ms": round(ms_i0, 4),
                                                       "i0": [float(v) for v in i0_dev.cpu()]}
        log(f"[bench] i0 estimate {res['extras']['i0_estimate']}")
        # the paper's percentile modes against the exact global histogram percentile
        med = torch.empty(2, dtype=torch.float32, device=dev)
        n_bands = (Hh + 1023) // 1024
        ws_b = S.workspace(S.workspace_size(S.OP_BAND_PERCENTILES, 0, n_bands, 0), dev)
        ms_band = timed(lambda: S.spcn_band_percentiles(img, w_fit, 1024, p, ws=ws_b), args.steps, args.warmup,
                        stream)
        med, _, _ = S.spcn_band_percentiles(img, w_fit, 1024, p, ws=ws_b)
        sp = torch.empty(2, dtype=torch.float32, device=dev)
        ws_s = S.workspace(S.workspace_size(S.OP_SAMPLE_PERCENTILE, 0, 0, n_samples), dev)
        ms_samp = timed(lambda: S.spcn_sample_percentile(img, w_fit, n_samples, 2024, p, p99_out=sp, ws=ws_s),
                        args.steps, args.warmup, stream)
        ex = torch.empty(2, dtype=torch.float32, device=dev)
        ws_x = S.workspace(S.workspace_size(S.OP_EXACT_PERCENTILE, 0, 0, 0), dev)
        ms_exact = timed(lambda: S.spcn_exact_percentile(img, w_fit, p, p99_out=ex, ws=ws_x), args.steps, args.warmup,
                         stream)
        del ws_x
        _, st_g = S.spcn_normalize(img, w_fit, w_tgt, scale_tgt, p, out=out)
        res["extras"]["percentile_modes"] = {
            "exact_order_statistic": [round(float(v), 5) for v in ex.cpu()], "exact_ms": round(ms_exact, 4),
            "global_hist": [round(float(v), 5) for v in st_g["p99_src"].cpu()],
            "band_median_1024_rows": [round(float(v), 5) for v in med.cpu()], "band_ms": round(ms_band, 4),
            "sample_200k": [round(float(v), 5) for v in sp.cpu()], "sample_ms": round(ms_samp, 4)}
        log(f"[bench] percentile modes {res['extras']['percentile_modes']}")
        # out-of-core: the first 8192 rows of the slide from pinned host memory, chunks of 512 rows
        rows = min(Hh, 8192)
        host = torch.empty((rows, Ww, 3), dtype=torch.uint8, pin_memory=True)
        host.copy_(img[:rows])
        host_out = torch.empty_like(host, pin_memory=True)
        ws_min = S.workspace_size(S.OP_STREAM_NORMALIZE, Ww, 512, 0)
        n_chunks = (rows + 511) // 512
        ws_all = ws_min + n_chunks * (((3 * 512 * Ww) + 255) // 256 * 256)   # every chunk resident
        cin, cout = torch.cuda.Stream(), torch.cuda.Stream()
        npx = rows * Ww
        # the link on its own: pinned host -> device and back, 1.2 GB each way, on a copy stream
        dbuf = torch.empty_like(host, device=dev)
        ms_h2d = timed(lambda: dbuf.copy_(host, non_blocking=True), 3, 1, stream)
        ms_d2h = timed(lambda: host_out.copy_(dbuf, non_blocking=True), 3, 1, stream)
        del dbuf
        h2d_peak, d2h_peak = 3 * npx / ms_h2d / 1e6, 3 * npx / ms_d2h / 1e6
        runs = {}
        for tag, wsb in (("minimal_workspace", ws_min), ("all_chunks_resident", ws_all)):
            ws_st = S.workspace(wsb, dev)
            ms_st = timed(lambda: S.spcn_normalize_streamed(host, w_fit, w_tgt, scale_tgt, p, chunk_rows=512,
                                                            host_out=host_out, ws=ws_st, copy_in=cin, copy_out=cout),
                          max(2, args.steps // 2), 1, stream)
            res_c = S.stream_resident_chunks(rows, Ww, 512, wsb)
            h2d_bytes = 3 * npx * (2 - res_c / n_chunks)    # resident chunks cross the link once
            runs[tag] = {"workspace_bytes": int(wsb), "resident_chunks": res_c, "chunks": n_chunks,
                         "resident_frac": round(res_c / n_chunks, 3), "ms": round(ms_st, 3),
                         "Mpx_s_pcie_inclusive": round(npx / ms_st / 1e3, 1),
                         "link_GBs_h2d": round(h2d_bytes / ms_st / 1e6, 1),
                         "link_GBs_d2h": round(3 * npx / ms_st / 1e6, 1),
                         "h2d_util": round(h2d_bytes / ms_st / 1e6 / h2d_peak, 3)}
            del ws_st
        res["extras"]["streamed_host_slide"] = {
            "rows": rows, "pixels": npx, "chunk_rows": 512, "copy_peak_GBs_h2d": round(h2d_peak, 1),
            "copy_peak_GBs_d2h": round(d2h_peak, 1), **runs}
        log(f"[bench] streamed {res['extras']['streamed_host_slide']}")
        del host, host_out
    if args.extras and args.workload == "slide":
        del img, out
        torch.cuda.empty_cache()
        extras = {}
        try:
            extras["densities_8192"] = bench_densities(dev, S, synth, args.steps, args.warmup)
            log(f"[bench] densities {extras['densities_8192']}")
        except Exception as e:   # report, never hide, a failing extra
            extras["densities_8192"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            extras["batched"] = bench_batched(dev, S, synth, args.steps, args.warmup, tune=args.autotune)
            log(f"[bench] batched {extras['batched']}")
        except Exception as e:   # report, never hide, a failing extra
            extras["batched"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        try:
            extras["fwd_bwd"] = bench_fwdbwd(dev, S, synth, args.steps, args.warmup)
            log(f"[bench] fwd_bwd {extras['fwd_bwd']}")
        except Exception as e:
            extras["fwd_bwd"] = {"error": repr(e)}
        res.setdefault("extras", {}).update(extras)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
