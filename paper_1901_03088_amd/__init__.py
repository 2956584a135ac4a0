"""Python binding of libspcn (include/spcn.h): SPCN colour normalisation on MI355X.

Argument marshalling only -- every step of the method runs in the HIP library.  Torch supplies
device memory and the current stream.  The functions keep the C names (spcn_densities,
spcn_normalize, ...) and take torch tensors; a few conveniences allocate the outputs.

The library must be built (``python -m paper_1901_03088_amd.build`` or ``__graft_entry__.build()``);
importing this package without it raises ImportError: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# SPCN_LIB: another build of the same sources (the sanitizer test loads an instrumented one)
LIB_PATH = os.environ.get("SPCN_LIB") or os.path.join(HERE, "libspcn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libspcn.so is not built ({LIB_PATH}); run paper_1901_03088_amd/build.py")
_L = C.CDLL(LIB_PATH)

# ------------------------------------------------------------------ ABI mirror

SPCN_OK, SPCN_E_ARG, SPCN_E_WORKSPACE, SPCN_E_HIP, SPCN_E_UNSUPPORTED = range(5)
FLAG_NO_TISSUE, FLAG_RANGE, FLAG_BIN0, FLAG_BASIS, FLAG_SHORT, FLAG_BATCH, FLAG_TIMEOUT, FLAG_NO_BACKGROUND, \
    FLAG_RANGE_RETRY, FLAG_SCALE = 1, 2, 4, 8, 16, 32, 64, 128, 256, 512
OP_DENSITIES, OP_NORMALIZE, OP_ESTIMATE_BASIS, OP_NORMALIZE_BATCHED, OP_ESTIMATE_BATCHED, \
    OP_FORWARD_F32, OP_BACKWARD_F32, OP_ESTIMATE_I0, OP_SAMPLE_PERCENTILE, OP_BAND_PERCENTILES, \
    OP_STREAM_NORMALIZE, OP_EXACT_PERCENTILE, OP_BANDWIDTH_PROBE = range(13)
HIST_BINS = 256
OPT_P1_VARIANT, OPT_P2_VARIANT, OPT_P2_BLOCKS_PER_CU, OPT_BATCH_CHUNK = range(4)


class spcn_params(C.Structure):
    _fields_ = [("i0", C.c_float * 3), ("lambda_", C.c_float), ("white_sum", C.c_int32),
                ("percentile", C.c_float), ("hist_hi", C.c_float * 2), ("hist_hi_dev", C.c_void_p),
                ("auto_range", C.c_int32)]


class spcn_norm_stats(C.Structure):
    _fields_ = [("hist", C.c_void_p), ("p99_src", C.c_void_p), ("scale", C.c_void_p), ("flags", C.c_void_p),
                ("hist_hi", C.c_void_p)]


class spcn_tile(C.Structure):
    _fields_ = [("src", C.c_void_p), ("out", C.c_void_p), ("height", C.c_int64), ("width", C.c_int64)]


_vp, _i64, _i32, _f, _u64, _sz = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_uint64, C.c_size_t
_P = C.POINTER(spcn_params)

_SIGS = {
    "spcn_default_params": (None, [_P]),
    "spcn_workspace_size": (_sz, [C.c_int, _i64, _i64, _i64]),
    "spcn_densities": (C.c_int, [_vp, _i64, _i64, _vp, _P, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_normalize": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp, C.POINTER(spcn_norm_stats), _vp,
                                 _sz, _vp]),
    "spcn_normalize_noalloc": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp,
                                         C.POINTER(spcn_norm_stats), _vp]),
    "spcn_recolor": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp, _vp, C.POINTER(spcn_norm_stats),
                               _vp]),
    "spcn_estimate_basis": (C.c_int, [_vp, _i64, _i64, _P, _f, _i64, _u64, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _sz, _vp]),
    "spcn_estimate_basis_batched": (C.c_int, [_vp, _i32, _i64, _P, _f, _i64, _u64, _i32, _vp, _vp, _vp, _vp,
                                              _vp, _vp, _sz, _vp]),
    "spcn_estimate_i0": (C.c_int, [_vp, _i64, _i64, _i64, _u64, _i32, _f, _vp, _vp, _vp, _sz, _vp]),
    "spcn_band_percentiles": (C.c_int, [_vp, _i64, _i64, _vp, _P, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_sample_percentile": (C.c_int, [_vp, _i64, _i64, _vp, _P, _i64, _u64, _vp, _vp, _vp, _sz, _vp]),
    "spcn_exact_percentile": (C.c_int, [_vp, _i64, _i64, _vp, _P, _vp, _vp, _vp, _sz, _vp]),
    "spcn_recolor_p99": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp, _vp, _vp, _vp, _vp]),
    "spcn_normalize_streamed": (C.c_int, [_vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _i64, _vp, _vp, _sz, _vp,
                                          _vp, _vp]),
    "spcn_stream_resident_chunks": (_i64, [_i64, _i64, _i64, _sz]),
    "spcn_normalize_batched": (C.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _P, _vp, _vp, _vp, _vp, _vp, _sz,
                                         _vp]),
    "spcn_normalize_f32": (C.c_int, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _P, _vp, _vp,
                                     _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_normalize_backward": (C.c_int, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _P, _vp,
                                          _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_bandwidth_probe": (C.c_int, [_vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "spcn_set_option": (C.c_int, [C.c_int, C.c_int]),
    "spcn_get_option": (C.c_int, [C.c_int]),
    "spcn_status_string": (C.c_char_p, [C.c_int]),
    "spcn_last_error": (C.c_char_p, []),
    "spcn_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_L, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


class SPCNError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _L.spcn_status_string(status).decode()
        detail = _L.spcn_last_error().decode()
        super().__init__(f"{where}: {msg}: {detail}")


def _check(status: int, where: str):
    if status != SPCN_OK:
        raise SPCNError(status, where)


def params(i0=(255.0, 255.0, 255.0), lam=0.01, white_sum=660, percentile=99.0, hist_hi=(4.0, 4.0),
           hist_hi_dev: torch.Tensor | None = None, auto_range: bool = True) -> spcn_params:
    """Parameters; hist_hi_dev is a device float32 tensor of ranges ([2], or [n_tiles, 2] for the
    batched normalisation) that replaces hist_hi (the struct keeps a reference to it)."""
    p = spcn_params()
    _L.spcn_default_params(C.byref(p))
    p.i0[:] = [float(v) for v in (i0 if hasattr(i0, "__len__") else (i0, i0, i0))]
    p.lambda_ = float(lam)
    p.white_sum = int(white_sum)
    p.percentile = float(percentile)
    p.hist_hi[:] = [float(v) for v in (hist_hi if hasattr(hist_hi, "__len__") else (hist_hi, hist_hi))]
    if hist_hi_dev is not None:
        _dev(hist_hi_dev, torch.float32, "hist_hi_dev")
        p.hist_hi_dev = hist_hi_dev.data_ptr()
        p._hist_hi_ref = hist_hi_dev
    p.auto_range = 1 if auto_range else 0
    return p


def copy_params(p: spcn_params, hist_hi_dev: torch.Tensor | None = None) -> spcn_params:
    """A copy of p; with hist_hi_dev, reading its range from that device tensor."""
    q = spcn_params()
    C.pointer(q)[0] = p
    if getattr(p, "_hist_hi_ref", None) is not None:
        q._hist_hi_ref = p._hist_hi_ref
    if hist_hi_dev is not None:
        _dev(hist_hi_dev, torch.float32, "hist_hi_dev")
        q.hist_hi_dev = hist_hi_dev.data_ptr()
        q._hist_hi_ref = hist_hi_dev
    return q


def workspace_size(op: int, n_px: int = 0, n_items: int = 0, n_samples: int = 0) -> int:
    return int(_L.spcn_workspace_size(op, n_px, n_items, n_samples))


def _dev(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace(nbytes: int, device) -> torch.Tensor:
    """Device workspace of at least nbytes (256-byte aligned, as the library requires)."""
    return torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)


def _ws_ptr(ws: torch.Tensor | None):
    if ws is None:
        return None, 0
    addr = ws.data_ptr()
    aligned = (addr + 255) & ~255
    return C.c_void_p(aligned), ws.numel() - (aligned - addr)


def as_basis(W, device) -> torch.Tensor:
    """3x2 matrix (columns = stains) or 6-vector -> device float32 [6] in column-major order."""
    t = torch.as_tensor(W, dtype=torch.float64)
    if t.shape == (3, 2):
        t = t.t().reshape(6)
    return t.reshape(6).to(torch.float32).to(device).contiguous()


# ------------------------------------------------------------------ entry points

def spcn_densities(img: torch.Tensor, w: torch.Tensor, p: spcn_params | None = None, want_h: bool = True,
                   h_out=None, hist_out=None, p99_out=None, flags_out=None, finalize: bool = True,
                   hist_hi_out=None, ws=None):
    """img (H, W, 3) uint8 on the GPU; w float32 [6].  Returns (h [2, H*W] or None, hist [2, 256]
    uint64, p99 [2] float32, flags [2] int32); with finalize=False no percentile is taken and
    p99 / flags are None.  hist_hi_out (device float32 [2]) receives the histogram's range."""
    _dev(img, torch.uint8, "img")
    _dev(w, torch.float32, "w")
    p = p or params()
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    n = H * W_
    if want_h and h_out is None:
        h_out = torch.empty((2, n), dtype=torch.float32, device=dev)
    hist_out = hist_out if hist_out is not None else torch.empty((2, HIST_BINS), dtype=torch.uint64, device=dev)
    if finalize:
        p99_out = p99_out if p99_out is not None else torch.empty(2, dtype=torch.float32, device=dev)
        flags_out = flags_out if flags_out is not None else torch.empty(2, dtype=torch.int32, device=dev)
    else:
        p99_out = flags_out = None
    if ws is None:
        ws = workspace(workspace_size(OP_DENSITIES), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_densities(_ptr(img), H, W_, _ptr(w), C.byref(p), _ptr(h_out if want_h else None),
                             _ptr(hist_out), _ptr(p99_out), _ptr(flags_out), _ptr(hist_hi_out), wsp, wsn, _stream()),
           "spcn_densities")
    return (h_out if want_h else None), hist_out, p99_out, flags_out


def spcn_normalize(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                   p: spcn_params | None = None, i0_out=None, out=None, stats: bool = True, ws=None):
    """src (H, W, 3) uint8 on the GPU.  Returns (out, dict(hist, p99_src, scale, flags, hist_hi))."""
    _dev(src, torch.uint8, "src")
    for t, nm in ((w_src, "w_src"), (w_tgt, "w_tgt"), (scale_tgt, "scale_tgt")):
        _dev(t, torch.float32, nm)
    p = p or params()
    H, W_ = int(src.shape[0]), int(src.shape[1])
    dev = src.device
    out = out if out is not None else torch.empty_like(src)
    st = None
    res = {}
    if stats:
        res = {"hist": torch.empty((2, HIST_BINS), dtype=torch.uint64, device=dev),
               "p99_src": torch.empty(2, dtype=torch.float32, device=dev),
               "scale": torch.empty(2, dtype=torch.float32, device=dev),
               "flags": torch.empty(2, dtype=torch.int32, device=dev),
               "hist_hi": torch.empty(2, dtype=torch.float32, device=dev)}
        st = spcn_norm_stats(res["hist"].data_ptr(), res["p99_src"].data_ptr(), res["scale"].data_ptr(),
                             res["flags"].data_ptr(), res["hist_hi"].data_ptr())
    if ws is None:
        ws = workspace(workspace_size(OP_NORMALIZE), dev)
    wsp, wsn = _ws_ptr(ws)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize(_ptr(src), H, W_, _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p),
                             _ptr(out), C.byref(st) if st is not None else None, wsp, wsn, _stream()),
           "spcn_normalize")
    return out, res


def spcn_normalize_noalloc(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                           out: torch.Tensor, p: spcn_params | None = None, i0_out=None, stats: dict | None = None):
    """spcn_normalize without a workspace (the library's static per-GPU scratch): out and the
    optional stats tensors (keys hist, p99_src, scale, flags, hist_hi; any may be missing) are
    the caller's, so the call allocates nothing."""
    _dev(src, torch.uint8, "src")
    _dev(out, torch.uint8, "out")
    for t, nm in ((w_src, "w_src"), (w_tgt, "w_tgt"), (scale_tgt, "scale_tgt")):
        _dev(t, torch.float32, nm)
    p = p or params()
    st = None
    if stats is not None:
        ptr = {k: (v.data_ptr() if v is not None else None) for k, v in stats.items()}
        st = spcn_norm_stats(ptr.get("hist"), ptr.get("p99_src"), ptr.get("scale"), ptr.get("flags"),
                             ptr.get("hist_hi"))
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize_noalloc(_ptr(src), int(src.shape[0]), int(src.shape[1]), _ptr(w_src), _ptr(w_tgt),
                                     _ptr(scale_tgt), io, C.byref(p), _ptr(out),
                                     C.byref(st) if st is not None else None, _stream()),
           "spcn_normalize_noalloc")
    return out


def spcn_recolor(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                 hist: torch.Tensor, p: spcn_params | None = None, i0_out=None, out=None, stats=True):
    """Pass 2 alone, from a given [2, 256] uint64 histogram.  Returns (out, dict(p99_src, scale, flags,
    hist_hi)); stats may be a dict of such preallocated device tensors to write into."""
    _dev(src, torch.uint8, "src")
    _dev(hist, torch.uint64, "hist")
    p = p or params()
    H, W_ = int(src.shape[0]), int(src.shape[1])
    dev = src.device
    out = out if out is not None else torch.empty_like(src)
    res = {}
    st = None
    if isinstance(stats, dict):
        res = stats
        st = spcn_norm_stats(None, res["p99_src"].data_ptr(), res["scale"].data_ptr(), res["flags"].data_ptr(),
                             res["hist_hi"].data_ptr())
    elif stats:
        res = {"p99_src": torch.empty(2, dtype=torch.float32, device=dev),
               "scale": torch.empty(2, dtype=torch.float32, device=dev),
               "flags": torch.empty(2, dtype=torch.int32, device=dev),
               "hist_hi": torch.empty(2, dtype=torch.float32, device=dev)}
        st = spcn_norm_stats(None, res["p99_src"].data_ptr(), res["scale"].data_ptr(), res["flags"].data_ptr(),
                             res["hist_hi"].data_ptr())
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_recolor(_ptr(src), H, W_, _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p),
                           _ptr(hist), _ptr(out), C.byref(st) if st is not None else None, _stream()),
           "spcn_recolor")
    return out, res


def spcn_estimate_basis(img: torch.Tensor, n_samples: int, seed: int, p: spcn_params | None = None,
                        lambda_nmf: float = 0.1, n_iter: int = 50, w_init=None, want_p99: bool = True,
                        w_out=None, ws=None, hist_hi_out=None):
    """Sparse-NMF stain basis of a uint8 (H, W, 3) image.  Returns (w [6] float32, sample_p99 [2]
    or None, flags [2] int32).  hist_hi_out (device float32 [2]) receives the histogram range derived
    from the sample percentile (feed it to params(hist_hi_dev=...))."""
    _dev(img, torch.uint8, "img")
    p = p or params()
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    w_out = w_out if w_out is not None else torch.empty(6, dtype=torch.float32, device=dev)
    sp = torch.empty(2, dtype=torch.float32, device=dev) if want_p99 else None
    flags = torch.empty(2, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_ESTIMATE_BASIS, H * W_, 1, n_samples), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_estimate_basis(_ptr(img), H, W_, C.byref(p), float(lambda_nmf), int(n_samples),
                                  int(seed) & (2 ** 64 - 1), int(n_iter), _ptr(w_init), _ptr(w_out), _ptr(sp),
                                  _ptr(hist_hi_out), _ptr(flags), wsp, wsn, _stream()), "spcn_estimate_basis")
    return w_out, sp, flags


def spcn_estimate_i0(img: torch.Tensor, n_samples: int = 100000, seed: int = 0, white_sum: int = 660,
                     percentile: float = 80.0, i0_out=None, ws=None):
    """Channel-wise background intensity of a uint8 (H, W, 3) image (Sec. 3.1 item 1).  Returns
    (i0 [3] float32 on the device, flags [1] int32).  Feed it back as params(i0=...) / i0_out."""
    _dev(img, torch.uint8, "img")
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    i0_out = i0_out if i0_out is not None else torch.empty(3, dtype=torch.float32, device=dev)
    flags = torch.empty(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_ESTIMATE_I0, 0, 0, n_samples), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_estimate_i0(_ptr(img), H, W_, int(n_samples), C.c_uint64(seed & (2**64 - 1)), int(white_sum),
                               float(percentile), _ptr(i0_out), _ptr(flags), wsp, wsn, _stream()), "spcn_estimate_i0")
    return i0_out, flags


def spcn_band_percentiles(img: torch.Tensor, w: torch.Tensor, band_rows: int, p: spcn_params | None = None,
                          ws=None):
    """Median over row bands of per-band percentiles.  Returns (median [2], band_p99 [n_bands, 2],
    flags [2]) on the device."""
    _dev(img, torch.uint8, "img"); _dev(w, torch.float32, "w")
    p = p or params()
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    nb = (H + band_rows - 1) // band_rows
    med = torch.empty(2, dtype=torch.float32, device=dev)
    bands = torch.empty((nb, 2), dtype=torch.float32, device=dev)
    flags = torch.empty(2, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_BAND_PERCENTILES, 0, nb, 0), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_band_percentiles(_ptr(img), H, W_, _ptr(w), C.byref(p), int(band_rows), _ptr(bands), _ptr(med),
                                    _ptr(flags), wsp, wsn, _stream()), "spcn_band_percentiles")
    return med, bands, flags


def spcn_sample_percentile(img: torch.Tensor, w: torch.Tensor, n_samples: int, seed: int,
                           p: spcn_params | None = None, p99_out=None, ws=None):
    """Percentile of the sub-sampled non-white pixels' densities.  Returns (p99 [2], flags [2])."""
    _dev(img, torch.uint8, "img"); _dev(w, torch.float32, "w")
    p = p or params()
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    p99_out = p99_out if p99_out is not None else torch.empty(2, dtype=torch.float32, device=dev)
    flags = torch.empty(2, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_SAMPLE_PERCENTILE, 0, 0, n_samples), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_sample_percentile(_ptr(img), H, W_, _ptr(w), C.byref(p), int(n_samples),
                                     C.c_uint64(seed & (2**64 - 1)), _ptr(p99_out), _ptr(flags), wsp, wsn, _stream()),
           "spcn_sample_percentile")
    return p99_out, flags


def spcn_exact_percentile(img: torch.Tensor, w: torch.Tensor, p: spcn_params | None = None, p99_out=None,
                          ws=None):
    """Exact nearest-rank percentile of the densities of all non-white pixels.  Returns (p99 [2], flags [2])."""
    _dev(img, torch.uint8, "img"); _dev(w, torch.float32, "w")
    p = p or params()
    H, W_ = int(img.shape[0]), int(img.shape[1])
    dev = img.device
    p99_out = p99_out if p99_out is not None else torch.empty(2, dtype=torch.float32, device=dev)
    flags = torch.empty(2, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_EXACT_PERCENTILE, 0, 0, 0), dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_exact_percentile(_ptr(img), H, W_, _ptr(w), C.byref(p), _ptr(p99_out), _ptr(flags), wsp, wsn,
                                    _stream()), "spcn_exact_percentile")
    return p99_out, flags


def spcn_recolor_p99(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                     p99_src: torch.Tensor, p: spcn_params | None = None, i0_out=None, out=None):
    """Pass 2 with given source percentiles (device [2]).  Returns (out, scale [2], flags [2])."""
    _dev(src, torch.uint8, "src"); _dev(p99_src, torch.float32, "p99_src")
    p = p or params()
    H, W_ = int(src.shape[0]), int(src.shape[1])
    out = out if out is not None else torch.empty_like(src)
    scale = torch.empty(2, dtype=torch.float32, device=src.device)
    flags = torch.empty(2, dtype=torch.int32, device=src.device)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_recolor_p99(_ptr(src), H, W_, _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p),
                               _ptr(p99_src), _ptr(out), _ptr(scale), _ptr(flags), _stream()), "spcn_recolor_p99")
    return out, scale, flags


def spcn_normalize_streamed(host_src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor,
                            scale_tgt: torch.Tensor, p: spcn_params | None = None, chunk_rows: int = 1024,
                            i0_out=None, host_out=None, ws=None, copy_in=None, copy_out=None):
    """Normalises a pinned host (H, W, 3) uint8 tensor through the device in row chunks.  Returns
    (host_out, dict(p99_src, scale, flags) on the device); host_out is complete once the current
    stream is."""
    if host_src.device.type != "cpu" or not host_src.is_pinned() or host_src.dtype != torch.uint8:
        raise ValueError("host_src must be a pinned CPU uint8 tensor")
    if not host_src.is_contiguous() or host_src.dim() != 3 or host_src.shape[2] != 3:
        raise ValueError("host_src must be a contiguous (H, W, 3) tensor")
    p = p or params()
    dev = w_src.device
    H, W_ = int(host_src.shape[0]), int(host_src.shape[1])
    host_out = host_out if host_out is not None else torch.empty_like(host_src, pin_memory=True)
    if ws is None:
        ws = workspace(workspace_size(OP_STREAM_NORMALIZE, W_, chunk_rows, 0), dev)
    wsp, wsn = _ws_ptr(ws)
    res = {"p99_src": torch.empty(2, dtype=torch.float32, device=dev),
           "scale": torch.empty(2, dtype=torch.float32, device=dev),
           "flags": torch.empty(2, dtype=torch.int32, device=dev)}
    st = spcn_norm_stats(0, res["p99_src"].data_ptr(), res["scale"].data_ptr(), res["flags"].data_ptr())
    copy_in = copy_in or torch.cuda.Stream(device=dev)
    copy_out = copy_out or copy_in
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize_streamed(C.c_void_p(host_src.data_ptr()), C.c_void_p(host_out.data_ptr()), H, W_,
                                      _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p), int(chunk_rows),
                                      C.byref(st), wsp, wsn, _stream(), C.c_void_p(copy_in.cuda_stream),
                                      C.c_void_p(copy_out.cuda_stream)), "spcn_normalize_streamed")
    return host_out, res


def stream_resident_chunks(height: int, width: int, chunk_rows: int, ws_bytes: int) -> int:
    """Chunks spcn_normalize_streamed keeps on the device between its passes with ws_bytes of workspace."""
    return int(_L.spcn_stream_resident_chunks(height, width, chunk_rows, ws_bytes))


def tile_table(srcs, outs=None) -> torch.Tensor:
    """Device array of spcn_tile descriptors for lists of (H, W, 3) uint8 tensors."""
    outs = outs if outs is not None else [None] * len(srcs)
    rows = []
    for s_, o_ in zip(srcs, outs):
        _dev(s_, torch.uint8, "tile")
        rows.append([s_.data_ptr(), 0 if o_ is None else o_.data_ptr(), int(s_.shape[0]), int(s_.shape[1])])
    t = torch.tensor(rows, dtype=torch.int64)
    return t.to(srcs[0].device)


def spcn_estimate_basis_batched(tiles: torch.Tensor, n_tiles: int, n_samples: int, seed: int,
                                p: spcn_params | None = None, lambda_nmf: float = 0.1, n_iter: int = 50,
                                w_init=None, want_p99: bool = True, ws=None, hist_hi_out=None):
    """Per-tile bases for a device tile table (see tile_table).  Returns (w [n, 6], p99 [n, 2] or None,
    flags [n, 2]).  hist_hi_out (device float32 [n, 2]) receives each tile's histogram range."""
    p = p or params()
    dev = tiles.device
    w_out = torch.empty((n_tiles, 6), dtype=torch.float32, device=dev)
    sp = torch.empty((n_tiles, 2), dtype=torch.float32, device=dev) if want_p99 else None
    flags = torch.empty((n_tiles, 2), dtype=torch.int32, device=dev)
    need = workspace_size(OP_ESTIMATE_BATCHED, 0, n_tiles, n_samples)
    if ws is None and need:
        ws = workspace(need, dev)
    wsp, wsn = _ws_ptr(ws)
    _check(_L.spcn_estimate_basis_batched(_ptr(tiles), int(n_tiles), 0, C.byref(p), float(lambda_nmf),
                                          int(n_samples), int(seed) & (2 ** 64 - 1), int(n_iter), _ptr(w_init),
                                          _ptr(w_out), _ptr(sp), _ptr(hist_hi_out), _ptr(flags), wsp, wsn, _stream()),
           "spcn_estimate_basis_batched")
    return w_out, sp, flags


def spcn_normalize_batched(tiles: torch.Tensor, n_tiles: int, total_px: int, w_src: torch.Tensor,
                           w_tgt: torch.Tensor, scale_tgt: torch.Tensor, p: spcn_params | None = None,
                           i0_out=None, ws=None, stats: bool = True, hist: bool = False):
    """Normalises every tile of a device tile table (tile_table(srcs, outs)), graph-capturable.
    w_src [n_tiles, 6].  Returns dict(p99 [n, 2], scale [n, 2], flags [n, 2]) (empty if stats=False),
    plus hist [n, 2, 256] uint64 when hist is True."""
    _dev(w_src, torch.float32, "w_src")
    p = p or params()
    dev = tiles.device
    res = {}
    if stats:
        res = {"p99": torch.empty((n_tiles, 2), dtype=torch.float32, device=dev),
               "scale": torch.empty((n_tiles, 2), dtype=torch.float32, device=dev),
               "flags": torch.empty((n_tiles, 2), dtype=torch.int32, device=dev)}
    if hist:
        res["hist"] = torch.empty((n_tiles, 2, HIST_BINS), dtype=torch.uint64, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_NORMALIZE_BATCHED, total_px, n_tiles), dev)
    wsp, wsn = _ws_ptr(ws)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize_batched(_ptr(tiles), int(n_tiles), int(total_px), _ptr(w_src), _ptr(w_tgt),
                                     _ptr(scale_tgt), io, C.byref(p), _ptr(res.get("p99")), _ptr(res.get("scale")),
                                     _ptr(res.get("flags")), _ptr(res.get("hist")), wsp, wsn, _stream()),
           "spcn_normalize_batched")
    return res


def spcn_bandwidth_probe(src: torch.Tensor, dst: torch.Tensor | None, mode: int, ws=None):
    """Bandwidth reference: mode 0 copies src's bytes into dst, mode 1 only reads them, both with the
    passes' streaming cache policy; modes 2 and 3 the same with the default policy."""
    n = src.numel() * src.element_size()
    if ws is None and mode in (1, 3):
        ws = workspace(workspace_size(OP_BANDWIDTH_PROBE), src.device)
    wsp, wsn = _ws_ptr(ws) if ws is not None else (None, 0)
    _check(_L.spcn_bandwidth_probe(_ptr(src), _ptr(dst), int(n), int(mode), wsp, wsn, _stream()),
           "spcn_bandwidth_probe")


def float_params(lam=0.01, white_sum=660, percentile=99.0) -> spcn_params:
    """Parameters of the float path: input in [0, 1], so i0 = 1."""
    return params(i0=(1.0, 1.0, 1.0), lam=lam, white_sum=white_sum, percentile=percentile)


def _per_sample(t, width, name):
    _dev(t, torch.float32, name)
    if t.dim() == 1:
        if t.numel() != width:
            raise ValueError(f"{name} must have {width} values or shape (n, {width})")
        return 0
    if t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{name} must have shape (n, {width})")
    return width


def spcn_normalize_f32(x: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                       p: spcn_params | None = None, i0_out=None, y=None, ws=None):
    """x (n, 3, H, W) float32 in [0, 1] on the GPU; w_src / w_tgt (n, 6) or (6,); scale_tgt (n, 2) or (2,).
    Returns (y, saved) with saved = dict(p99, scale, sel, flags), each (n, 2)."""
    _dev(x, torch.float32, "x")
    if x.dim() != 4 or x.shape[1] != 3:
        raise ValueError("x must have shape (n, 3, H, W)")
    n, _, H, W_ = (int(v) for v in x.shape)
    sw, st_, ss = _per_sample(w_src, 6, "w_src"), _per_sample(w_tgt, 6, "w_tgt"), _per_sample(scale_tgt, 2, "scale_tgt")
    p = p or float_params()
    dev = x.device
    y = y if y is not None else torch.empty_like(x)
    saved = {"p99": torch.empty((n, 2), dtype=torch.float32, device=dev),
             "scale": torch.empty((n, 2), dtype=torch.float32, device=dev),
             "sel": torch.empty((n, 2), dtype=torch.int64, device=dev),
             "flags": torch.empty((n, 2), dtype=torch.int32, device=dev)}
    if ws is None:
        ws = workspace(workspace_size(OP_FORWARD_F32, H * W_, n), dev)
    wsp, wsn = _ws_ptr(ws)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize_f32(_ptr(x), n, H, W_, _ptr(w_src), sw, _ptr(w_tgt), st_, _ptr(scale_tgt), ss, io,
                                 C.byref(p), _ptr(y), _ptr(saved["p99"]), _ptr(saved["scale"]), _ptr(saved["sel"]),
                                 _ptr(saved["flags"]), wsp, wsn, _stream()), "spcn_normalize_f32")
    return y, saved


def spcn_normalize_backward(x: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                            saved: dict, grad_y: torch.Tensor, p: spcn_params | None = None, i0_out=None, ws=None):
    """Adjoint of spcn_normalize_f32.  Returns (grad_x, grad_w_tgt, grad_scale): per sample ((n, 6), (n, 2))
    for per-sample parameters, or ((6,), (2,)) summed over the batch (by the library) for shared ones."""
    _dev(x, torch.float32, "x")
    _dev(grad_y, torch.float32, "grad_y")
    n, _, H, W_ = (int(v) for v in x.shape)
    sw, st_, ss = _per_sample(w_src, 6, "w_src"), _per_sample(w_tgt, 6, "w_tgt"), _per_sample(scale_tgt, 2, "scale_tgt")
    p = p or float_params()
    dev = x.device
    gx = torch.empty_like(x)
    gw = torch.empty((n, 6) if st_ else (6,), dtype=torch.float32, device=dev)
    gs = torch.empty((n, 2) if ss else (2,), dtype=torch.float32, device=dev)
    if ws is None:
        ws = workspace(workspace_size(OP_BACKWARD_F32, H * W_, n), dev)
    wsp, wsn = _ws_ptr(ws)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize_backward(_ptr(x), n, H, W_, _ptr(w_src), sw, _ptr(w_tgt), st_, _ptr(scale_tgt), ss, io,
                                      C.byref(p), _ptr(saved["p99"]), _ptr(saved["sel"]), _ptr(saved["flags"]),
                                      _ptr(grad_y), _ptr(gx), _ptr(gw), _ptr(gs), wsp, wsn, _stream()),
           "spcn_normalize_backward")
    return gx, gw, gs


class SPCNNormalize(torch.autograd.Function):
    """y = SPCN(x; W_src, W_tgt, scale_tgt) on float images, differentiable in x, W_tgt and scale_tgt
    (W_src is treated as a constant).  Shapes as in spcn_normalize_f32; a (6,) W_tgt or (2,) scale
    shared by the batch receives the sum of the per-sample gradients (summed by the library)."""

    @staticmethod
    def forward(ctx, x, w_src, w_tgt, scale_tgt, p=None, i0_out=None):
        x = x.contiguous()
        w_src, w_tgt, scale_tgt = w_src.contiguous(), w_tgt.contiguous(), scale_tgt.contiguous()
        y, saved = spcn_normalize_f32(x, w_src, w_tgt, scale_tgt, p, i0_out)
        ctx.save_for_backward(x, w_src, w_tgt, scale_tgt, saved["p99"], saved["sel"], saved["flags"])
        ctx.p, ctx.i0_out = p, i0_out
        return y

    @staticmethod
    def backward(ctx, gy):
        x, w_src, w_tgt, scale_tgt, p99, sel, flags = ctx.saved_tensors
        gx, gw, gs = spcn_normalize_backward(x, w_src, w_tgt, scale_tgt, {"p99": p99, "sel": sel, "flags": flags},
                                             gy.contiguous(), ctx.p, ctx.i0_out)
        return gx, None, gw, gs, None, None


def set_option(opt: int, value: int) -> None:
    _check(_L.spcn_set_option(int(opt), int(value)), "spcn_set_option")


def get_option(opt: int) -> int:
    return int(_L.spcn_get_option(int(opt)))


def version() -> str:
    return _L.spcn_version().decode()
