"""Seeded synthetic H&E-like inputs shared by the tests, the smoke check and the benchmark.

This module only *makes inputs*.  It holds none of the normalization method's arithmetic (no
optical-density transform of an input, no density solve, no percentile, no reconstruction) and
imports neither the oracle nor the HIP library.  Images are synthesised from known stain vectors
and known densities with a Beer-Lambert imaging model, then noised and quantised to uint8.

Recipe (stated again in the design doc):
  * stains: hematoxylin-like [0.65, 0.70, 0.29] and eosin-like [0.07, 0.99, 0.11], unit length,
    each rotated by an angle ~ U[-d, d] degrees towards a random unit vector orthogonal to it,
    clamped at 0 and renormalised (d = 5 for sources, 10 for the augmentation targets);
  * densities: two N(0,1) fields smoothed with a Gaussian of sigma = 8 px and standardised; the
    larger of the two picks the dominant stain; dominant density = D_j * Phi(z) with D_j ~ U[0.5,
    2.5] per image and stain; the other stain gets U[0, 0.15] of the dominant one per pixel;
  * background: a field smoothed with sigma = 32 px, the lowest `bg_frac` quantile is background,
    whose channels are i.i.d. integers U{235..255};
  * tissue pixels are 255 * exp(-W h) per channel; every pixel gets N(0, 2^2) noise, then rint and
    clamp to [0, 255].
Smoothed fields are drawn on a grid 4x (sigma 8) or 8x (sigma 32) coarser, blurred there with the
correspondingly smaller sigma, and bilinearly upsampled: same correlation length, far less work.
"""
from __future__ import annotations

import math
import numpy as np
import torch
import torch.nn.functional as F

H_REF = np.array([0.65, 0.70, 0.29])
E_REF = np.array([0.07, 0.99, 0.11])


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def reference_basis() -> np.ndarray:
    """Unit hematoxylin / eosin reference vectors as a 3x2 float64 matrix (columns = stains)."""
    return np.stack([unit(H_REF), unit(E_REF)], axis=1)


def jitter_column(rng: np.random.Generator, w, max_deg: float) -> np.ndarray:
    w = unit(w)
    u = rng.standard_normal(3)
    u -= u.dot(w) * w
    u = unit(u)
    th = math.radians(rng.uniform(-max_deg, max_deg))
    v = math.cos(th) * w + math.sin(th) * u
    v = np.maximum(v, 0.0)
    return unit(v)


def jitter_basis(rng: np.random.Generator, max_deg: float = 5.0, base: np.ndarray | None = None) -> np.ndarray:
    base = reference_basis() if base is None else np.asarray(base, dtype=np.float64)
    return np.stack([jitter_column(rng, base[:, 0], max_deg), jitter_column(rng, base[:, 1], max_deg)], axis=1)


def basis_f32(W: np.ndarray) -> np.ndarray:
    """3x2 basis -> float32 array of 6 in column-major order W[c + 3 j] (the library's layout)."""
    return np.ascontiguousarray(np.asarray(W, dtype=np.float64).T.reshape(6).astype(np.float32))


def _gauss_kernel(sigma: float, device) -> torch.Tensor:
    r = max(1, int(math.ceil(4.0 * sigma)))
    x = torch.arange(-r, r + 1, dtype=torch.float32, device=device)
    k = torch.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _blur_circular(z: torch.Tensor, sigma: float) -> torch.Tensor:
    """Separable Gaussian blur of a 2-D field with wrap-around borders."""
    k = _gauss_kernel(sigma, z.device)
    r = (k.numel() - 1) // 2
    x = z[None, None]
    x = F.pad(x, (r, r, 0, 0), mode="circular")
    x = F.conv2d(x, k.view(1, 1, 1, -1))
    x = F.pad(x, (0, 0, r, r), mode="circular")
    x = F.conv2d(x, k.view(1, 1, -1, 1))
    return x[0, 0]


def smooth_field(gen: torch.Generator, h: int, w: int, sigma: float, coarse: int) -> torch.Tensor:
    """Standardised Gaussian-smoothed white noise of correlation length sigma (pixels), drawn on a
    grid `coarse` times coarser and bilinearly upsampled."""
    dev = gen.device
    r = max(1, int(math.ceil(4.0 * sigma / coarse)))
    hc, wc = max(-(-h // coarse) + 2, 2 * r + 2), max(-(-w // coarse) + 2, 2 * r + 2)
    z = torch.randn((hc, wc), generator=gen, device=dev, dtype=torch.float32)
    z = _blur_circular(z, sigma / coarse)
    f = F.interpolate(z[None, None], scale_factor=coarse, mode="bilinear", align_corners=False)[0, 0]
    f = f[coarse:coarse + h, coarse:coarse + w]
    sub = f.reshape(-1)[:: 7]
    f = (f - sub.mean()) / sub.std().clamp_min(1e-12)
    return f.contiguous()


def densities(gen: torch.Generator, h: int, w: int, sigma: float = 8.0) -> torch.Tensor:
    """Two-stain density field with one dominant stain per pixel; returns (2, h, w) float32."""
    dev = gen.device
    z0 = smooth_field(gen, h, w, sigma, 4)
    z1 = smooth_field(gen, h, w, sigma, 4)
    D = 0.5 + 2.0 * torch.rand(2, generator=gen, device=dev, dtype=torch.float64)
    dom0 = z0 >= z1
    hd = torch.special.ndtr(torch.where(dom0, z0, z1))
    frac = torch.rand((h, w), generator=gen, device=dev, dtype=torch.float32) * 0.15
    d0, d1 = float(D[0]), float(D[1])
    H = torch.empty((2, h, w), dtype=torch.float32, device=dev)
    H[0] = torch.where(dom0, d0 * hd, d1 * hd * frac)
    H[1] = torch.where(dom0, d0 * hd * frac, d1 * hd)
    return H


def background_mask(gen: torch.Generator, h: int, w: int, bg_frac: float) -> torch.Tensor:
    if bg_frac <= 0:
        return torch.zeros((h, w), dtype=torch.bool, device=gen.device)
    f = smooth_field(gen, h, w, 32.0, 8)
    sub = f.reshape(-1)[:: 13]
    k = max(1, int(round(bg_frac * sub.numel())))
    thr = torch.kthvalue(sub.cpu(), k).values.item()
    return f < thr


def render(gen: torch.Generator, W: np.ndarray, H: torch.Tensor, bg: torch.Tensor, noise: float = 2.0) -> torch.Tensor:
    """Beer-Lambert imaging of densities H (2,h,w) through stains W (3x2), plus background and
    noise; returns (h, w, 3) uint8."""
    dev = gen.device
    h, w = H.shape[1:]
    I = torch.empty((h, w, 3), dtype=torch.float32, device=dev)
    for c in range(3):
        od = float(W[c, 0]) * H[0] + float(W[c, 1]) * H[1]
        I[:, :, c] = torch.exp(-od) * 255.0
    bgv = torch.randint(235, 256, (h, w, 3), generator=gen, device=dev, dtype=torch.int32).to(torch.float32)
    I = torch.where(bg[:, :, None], bgv, I)
    if noise > 0:
        I += torch.randn((h, w, 3), generator=gen, device=dev, dtype=torch.float32) * noise
    return torch.round(I).clamp_(0, 255).to(torch.uint8)


def make_image(seed: int, h: int, w: int, bg_frac: float = 0.3, max_deg: float = 5.0,
               W: np.ndarray | None = None, noise: float = 2.0, device="cpu", keep_h: bool = False):
    """One seeded synthetic image.  Returns dict(img (h,w,3) uint8 tensor on `device`, W 3x2
    float64 numpy, and with keep_h the true densities H (2,h,w) and background mask)."""
    rng = np.random.default_rng(seed)
    if W is None:
        W = jitter_basis(rng, max_deg)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 7919 + 17)
    H = densities(gen, h, w)
    bg = background_mask(gen, h, w, bg_frac)
    img = render(gen, W, H, bg, noise)
    out = {"img": img, "W": np.asarray(W, dtype=np.float64)}
    if keep_h:
        out["H"] = H
        out["bg"] = bg
    return out


# ------------------------------------------------------------------ named workloads

def config0(size: int = 1024, device="cpu"):
    """Plain case: one source (seed 0) and one target (seed 1) image, 1024 x 1024 by default."""
    return make_image(0, size, size, device=device), make_image(1, size, size, device=device)


def target_image(size: int = 1024, device="cpu"):
    """The target image every workload normalises to (seed 1)."""
    return make_image(1, size, size, device=device)


def config1(size: int = 8192, device="cpu"):
    """Single large image (8192 x 8192 = 67 Mpixel by default), seed 10."""
    return make_image(10, size, size, device=device)


SLIDE_H, SLIDE_W, SLIDE_BLOCK = 40000, 50000, 4096


def slide_layout(seed: int = 20, height: int = SLIDE_H, width: int = SLIDE_W, block: int = SLIDE_BLOCK,
                 tissue_slot_frac: float = 0.57):
    """Slot plan of the gigapixel slide: a grid of block-sized slots, each tissue or background,
    cropped at the slide edge.  Returns a list of (y0, x0, hh, ww, tissue) tuples.  With 30%
    background inside tissue slots and 57% tissue slots, ~60% of the slide is background."""
    rng = np.random.default_rng(seed)
    rows, cols = -(-height // block), -(-width // block)
    plan = []
    for r in range(rows):
        for c in range(cols):
            y0, x0 = r * block, c * block
            hh, ww = min(block, height - y0), min(block, width - x0)
            plan.append((y0, x0, hh, ww, bool(rng.uniform() < tissue_slot_frac)))
    return plan


def slide_basis(seed: int = 20) -> np.ndarray:
    """The stain basis of the slide (one slide, one staining)."""
    return jitter_basis(np.random.default_rng(seed + 1000), 5.0)


def slot_image(plan, k: int, W: np.ndarray, seed: int = 20, device="cpu") -> torch.Tensor:
    """Pixels (hh, ww, 3) uint8 of slot k: a field of its own seed (seed * 1000 + k), tissue with
    30% background blobs, or all background."""
    y0, x0, hh, ww, tissue = plan[k]
    return make_image(seed * 1000 + k, hh, ww, bg_frac=0.3 if tissue else 1.0, W=W, device=device)["img"]


def make_slide(seed: int = 20, height: int = SLIDE_H, width: int = SLIDE_W, block: int = SLIDE_BLOCK, device="cpu"):
    """The (height, width, 3) uint8 slide, every slot drawn from its own seeded field on `device`.
    Returns (img, W, plan)."""
    plan = slide_layout(seed, height, width, block)
    W = slide_basis(seed)
    out = torch.empty((height, width, 3), dtype=torch.uint8, device=device)
    for k, (y0, x0, hh, ww, _) in enumerate(plan):
        out[y0:y0 + hh, x0:x0 + ww] = slot_image(plan, k, W, seed, device)
    return out, W, plan


def tile_shapes(n_tiles: int = 512, seed: int = 30000, lo: int = 256, hi: int = 2048, step: int = 64):
    """Tile (height, width) pairs, each side uniform over lo..hi in steps of `step`."""
    rng = np.random.default_rng(seed)
    vals = np.arange(lo, hi + 1, step)
    return [(int(rng.choice(vals)), int(rng.choice(vals))) for _ in range(n_tiles)]


def make_tile(t: int, h: int, w: int, device="cpu"):
    """Tile t of the batched workload: its own jittered basis, seed 30000 + t."""
    return make_image(30000 + t, h, w, device=device)


def target_bases(n: int, seed: int = 40, max_deg: float = 10.0, base: np.ndarray | None = None):
    """Per-sample target bases for augmentation, each column jittered by up to max_deg degrees."""
    rng = np.random.default_rng(seed)
    return [jitter_basis(rng, max_deg, base) for _ in range(n)]


def float_batch(n: int = 64, size: int = 512, seed: int = 40, device="cpu"):
    """Differentiable workload: n images (n, 3, size, size) float32 in [0, 1] from the plain
    generator, their source bases, per-sample target bases jittered by up to 10 degrees around
    the target image's basis, and seeded loss weights U[0, 1)."""
    x = torch.empty((n, 3, size, size), dtype=torch.float32, device=device)
    Ws = []
    for i in range(n):
        d = make_image(seed * 1000 + i, size, size, device=device)
        x[i] = d["img"].permute(2, 0, 1).to(torch.float32) / 255.0
        Ws.append(d["W"])
    Wt = target_bases(n, seed, 10.0, make_image(1, 8, 8)["W"])
    gen = torch.Generator(device=device)
    gen.manual_seed(seed * 31 + 5)
    wts = torch.rand(x.shape, generator=gen, device=device, dtype=torch.float32)
    return x, Ws, Wt, wts
