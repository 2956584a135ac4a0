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
LIB_PATH = os.path.join(HERE, "libspcn.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libspcn.so is not built ({LIB_PATH}); run paper_1901_03088_amd/build.py")
_L = C.CDLL(LIB_PATH)

# ------------------------------------------------------------------ ABI mirror

SPCN_OK, SPCN_E_ARG, SPCN_E_WORKSPACE, SPCN_E_HIP, SPCN_E_UNSUPPORTED = range(5)
FLAG_NO_TISSUE, FLAG_RANGE, FLAG_BIN0, FLAG_BASIS, FLAG_SHORT = 1, 2, 4, 8, 16
OP_DENSITIES, OP_NORMALIZE, OP_ESTIMATE_BASIS, OP_NORMALIZE_BATCHED, OP_ESTIMATE_BATCHED, \
    OP_FORWARD_F32, OP_BACKWARD_F32 = range(7)
HIST_BINS = 256


class spcn_params(C.Structure):
    _fields_ = [("i0", C.c_float * 3), ("lambda_", C.c_float), ("white_sum", C.c_int32),
                ("percentile", C.c_float), ("hist_hi", C.c_float * 2)]


class spcn_norm_stats(C.Structure):
    _fields_ = [("hist", C.c_void_p), ("p99_src", C.c_void_p), ("scale", C.c_void_p), ("flags", C.c_void_p)]


class spcn_tile(C.Structure):
    _fields_ = [("src", C.c_void_p), ("out", C.c_void_p), ("height", C.c_int64), ("width", C.c_int64)]


_vp, _i64, _i32, _f, _u64, _sz = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_uint64, C.c_size_t
_P = C.POINTER(spcn_params)

_SIGS = {
    "spcn_default_params": (None, [_P]),
    "spcn_workspace_size": (_sz, [C.c_int, _i64, _i64, _i64]),
    "spcn_densities": (C.c_int, [_vp, _i64, _i64, _vp, _P, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_normalize": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp, C.POINTER(spcn_norm_stats), _vp,
                                 _sz, _vp]),
    "spcn_recolor": (C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _P, _vp, _vp, C.POINTER(spcn_norm_stats),
                               _vp]),
    "spcn_estimate_basis": (C.c_int, [_vp, _i64, _i64, _P, _f, _i64, _u64, _i32, _vp, _vp, _vp, _vp, _vp, _sz,
                                      _vp]),
    "spcn_estimate_basis_batched": (C.c_int, [_vp, _i32, _i64, _P, _f, _i64, _u64, _i32, _vp, _vp, _vp, _vp,
                                              _vp, _sz, _vp]),
    "spcn_normalize_batched": (C.c_int, [_vp, _i32, _i64, _vp, _vp, _vp, _vp, _P, _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_normalize_f32": (C.c_int, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _P, _vp, _vp,
                                     _vp, _vp, _vp, _vp, _sz, _vp]),
    "spcn_normalize_backward": (C.c_int, [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _P, _vp,
                                          _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
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


def params(i0=(255.0, 255.0, 255.0), lam=0.01, white_sum=660, percentile=99.0, hist_hi=(4.0, 4.0)) -> spcn_params:
    p = spcn_params()
    _L.spcn_default_params(C.byref(p))
    p.i0[:] = [float(v) for v in (i0 if hasattr(i0, "__len__") else (i0, i0, i0))]
    p.lambda_ = float(lam)
    p.white_sum = int(white_sum)
    p.percentile = float(percentile)
    p.hist_hi[:] = [float(v) for v in (hist_hi if hasattr(hist_hi, "__len__") else (hist_hi, hist_hi))]
    return p


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
                   h_out=None, hist_out=None, p99_out=None, flags_out=None, finalize: bool = True):
    """img (H, W, 3) uint8 on the GPU; w float32 [6].  Returns (h [2, H*W] or None, hist [2, 256]
    uint64, p99 [2] float32, flags [2] int32); with finalize=False no percentile is taken and
    p99 / flags are None."""
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
    _check(_L.spcn_densities(_ptr(img), H, W_, _ptr(w), C.byref(p), _ptr(h_out if want_h else None),
                             _ptr(hist_out), _ptr(p99_out), _ptr(flags_out), None, 0, _stream()), "spcn_densities")
    return (h_out if want_h else None), hist_out, p99_out, flags_out


def spcn_normalize(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                   p: spcn_params | None = None, i0_out=None, out=None, stats: bool = True, ws=None):
    """src (H, W, 3) uint8 on the GPU.  Returns (out, dict(hist, p99_src, scale, flags))."""
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
               "flags": torch.empty(2, dtype=torch.int32, device=dev)}
        st = spcn_norm_stats(res["hist"].data_ptr(), res["p99_src"].data_ptr(), res["scale"].data_ptr(),
                             res["flags"].data_ptr())
    if ws is None and not stats:
        ws = workspace(workspace_size(OP_NORMALIZE, H * W_), dev)
    wsp, wsn = _ws_ptr(ws)
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_normalize(_ptr(src), H, W_, _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p),
                             _ptr(out), C.byref(st) if st is not None else None, wsp, wsn, _stream()),
           "spcn_normalize")
    return out, res


def spcn_recolor(src: torch.Tensor, w_src: torch.Tensor, w_tgt: torch.Tensor, scale_tgt: torch.Tensor,
                 hist: torch.Tensor, p: spcn_params | None = None, i0_out=None, out=None, stats: bool = True):
    """Pass 2 alone, from a given [2, 256] uint64 histogram.  Returns (out, dict(p99_src, scale, flags))."""
    _dev(src, torch.uint8, "src")
    _dev(hist, torch.uint64, "hist")
    p = p or params()
    H, W_ = int(src.shape[0]), int(src.shape[1])
    dev = src.device
    out = out if out is not None else torch.empty_like(src)
    res = {}
    st = None
    if stats:
        res = {"p99_src": torch.empty(2, dtype=torch.float32, device=dev),
               "scale": torch.empty(2, dtype=torch.float32, device=dev),
               "flags": torch.empty(2, dtype=torch.int32, device=dev)}
        st = spcn_norm_stats(None, res["p99_src"].data_ptr(), res["scale"].data_ptr(), res["flags"].data_ptr())
    io = None if i0_out is None else (C.c_float * 3)(*[float(v) for v in i0_out])
    _check(_L.spcn_recolor(_ptr(src), H, W_, _ptr(w_src), _ptr(w_tgt), _ptr(scale_tgt), io, C.byref(p),
                           _ptr(hist), _ptr(out), C.byref(st) if st is not None else None, _stream()),
           "spcn_recolor")
    return out, res


def spcn_estimate_basis(img: torch.Tensor, n_samples: int, seed: int, p: spcn_params | None = None,
                        lambda_nmf: float = 0.1, n_iter: int = 50, w_init=None, want_p99: bool = True,
                        w_out=None, ws=None):
    """Sparse-NMF stain basis of a uint8 (H, W, 3) image.  Returns (w [6] float32, sample_p99 [2]
    or None, flags [2] int32)."""
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
                                  _ptr(flags), wsp, wsn, _stream()), "spcn_estimate_basis")
    return w_out, sp, flags


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
                                w_init=None, want_p99: bool = True, ws=None):
    """Per-tile bases for a device tile table (see tile_table).  Returns (w [n, 6], p99 [n, 2] or None,
    flags [n, 2])."""
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
                                          _ptr(w_out), _ptr(sp), _ptr(flags), wsp, wsn, _stream()),
           "spcn_estimate_basis_batched")
    return w_out, sp, flags


def version() -> str:
    return _L.spcn_version().decode()
