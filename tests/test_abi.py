"""CPU tests of the C-ABI boundary: the library loads, exports every function include/spcn.h declares,
and rejects invalid arguments on the host before anything reaches a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "spcn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spcn_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1901_03088_amd as s
    return s


def test_header_functions_all_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib._L, n), n
    assert set(names) == set(lib.EXPORTED)


def test_defaults_follow_the_paper(lib):
    """Library defaults against the constants the paper fixes (tests/golden/paper_constants.json)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    p = lib.params()
    assert list(p.i0) == [float(g["eq1_max_intensity_8bit"]["value"])] * 3
    assert p.white_sum == 3 * g["white_intensity_threshold"]["value"]      # mean of the three channels
    assert p.percentile == float(g["normalisation_percentile"]["value"])
    assert lib.workspace_size(lib.OP_ESTIMATE_I0, 0, 0, g["i0_max_samples"]["value"]) > 0   # the paper's cap fits
    import inspect
    sig = inspect.signature(lib.spcn_estimate_i0).parameters
    assert sig["n_samples"].default == g["i0_max_samples"]["value"]
    assert sig["percentile"].default == float(g["i0_percentile"]["value"])
    assert sig["white_sum"].default == 3 * g["background_intensity_threshold"]["value"]
    q = lib.spcn_params()
    lib._L.spcn_default_params(C.byref(q))
    assert list(q.hist_hi) == [4.0, 4.0]
    assert q.hist_hi_dev is None and q.auto_range == 1


def test_status_strings(lib):
    for s in range(5):
        assert lib._L.spcn_status_string(s)
    assert lib.version().startswith("spcn")


def call_normalize(lib, **kw):
    p = kw.pop("p", lib.params())
    args = dict(src=C.c_void_p(1 << 20), h=8, w=8, ws=C.c_void_p(1 << 24), wt=C.c_void_p(1 << 24),
                sc=C.c_void_p(1 << 24), out=C.c_void_p(2 << 20), wsp=C.c_void_p(3 << 20), wsn=1 << 20)
    args.update(kw)
    return lib._L.spcn_normalize(args["src"], args["h"], args["w"], args["ws"], args["wt"], args["sc"], None,
                                 C.byref(p), args["out"], None, args["wsp"], args["wsn"], None)


@pytest.mark.parametrize("kw,frag", [
    (dict(src=None), "src is NULL"),
    (dict(out=None), "out is NULL"),
    (dict(h=0), "height and width"),
    (dict(w=-3), "height and width"),
    (dict(src=C.c_void_p((1 << 20) + 1)), "aligned"),
    (dict(ws=None), "non-NULL"),
    (dict(out=C.c_void_p((1 << 20) + 96)), "overlap"),
    (dict(wsp=None), "workspace"),
    (dict(wsn=16), "workspace"),
    (dict(h=1 << 20, w=1 << 20), "2^36"),
])
def test_normalize_rejects(lib, kw, frag):
    st = call_normalize(lib, **kw)
    assert st in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
    assert frag in lib._L.spcn_last_error().decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(src=None), "src is NULL"),
    (dict(ws=None), "non-NULL"),
    (dict(out=C.c_void_p((1 << 20) + 96)), "overlap"),
    (dict(h=1 << 20, w=1 << 20), "2^36"),
])
def test_normalize_noalloc_rejects(lib, kw, frag):
    """The allocation-free entry point checks its arguments on the host, before it touches the
    device (no GPU here: a check that reached the device would report a HIP error instead)."""
    p = kw.pop("p", lib.params())
    args = dict(src=C.c_void_p(1 << 20), h=8, w=8, ws=C.c_void_p(1 << 24), wt=C.c_void_p(1 << 24),
                sc=C.c_void_p(1 << 24), out=C.c_void_p(2 << 20))
    args.update(kw)
    st = lib._L.spcn_normalize_noalloc(args["src"], args["h"], args["w"], args["ws"], args["wt"], args["sc"], None,
                                       C.byref(p), args["out"], None, None)
    assert st == lib.SPCN_E_ARG
    assert frag in lib._L.spcn_last_error().decode()


@pytest.mark.parametrize("field,value,frag", [
    ("lambda_", -0.1, "lambda"),
    ("lambda_", float("nan"), "lambda"),
    ("percentile", 0.0, "percentile"),
    ("percentile", 100.5, "percentile"),
    ("hist_hi", (3.0, 4.0), "power of two"),
    ("hist_hi", (4.0, 1024.0), "power of two"),
    ("i0", (255.0, 0.0, 255.0), "i0"),
    ("auto_range", 2, "auto_range"),
    ("hist_hi_dev", (1 << 24) + 2, "hist_hi_dev"),
])
def test_params_rejected(lib, field, value, frag):
    p = lib.params()
    if isinstance(value, tuple):
        getattr(p, field)[:] = list(value)
    else:
        setattr(p, field, value)
    st = call_normalize(lib, p=p)
    assert st == lib.SPCN_E_ARG
    assert frag in lib._L.spcn_last_error().decode()


def test_densities_requires_histogram(lib):
    p = lib.params()
    st = lib._L.spcn_densities(C.c_void_p(1 << 20), 4, 4, C.c_void_p(1 << 24), C.byref(p), None, None, None, None,
                               None, None, 0, None)
    assert st == lib.SPCN_E_ARG
    assert "hist_out" in lib._L.spcn_last_error().decode()


def test_densities_requires_workspace(lib):
    """The range and retry words of the histogram live in the workspace."""
    p = lib.params()
    st = lib._L.spcn_densities(C.c_void_p(1 << 20), 4, 4, C.c_void_p(1 << 24), C.byref(p), None, C.c_void_p(1 << 24),
                               None, None, None, None, 0, None)
    assert st == lib.SPCN_E_WORKSPACE


def test_workspace_sizes(lib):
    assert lib.workspace_size(lib.OP_NORMALIZE, 1000) >= 2 * 256 * 8
    assert lib.workspace_size(99, 10) == 0
    assert lib.workspace_size(lib.OP_NORMALIZE, -1) == 0


def test_options_ranges(lib):
    """Tuning options: defaults, accepted ranges, rejection of unknown options and bad values."""
    saved = [lib.get_option(o) for o in range(4)]
    assert saved == [6, 3, 8, 15]
    try:
        for opt, lo, hi in ((lib.OPT_P1_VARIANT, 0, 9), (lib.OPT_P2_VARIANT, 0, 5),
                            (lib.OPT_P2_BLOCKS_PER_CU, 1, 16), (lib.OPT_BATCH_CHUNK, 12, 18)):
            for v in (lo, hi):
                lib.set_option(opt, v)
                assert lib.get_option(opt) == v
            assert lib._L.spcn_set_option(opt, lo - 1) == lib.SPCN_E_ARG
            assert lib._L.spcn_set_option(opt, hi + 1) == lib.SPCN_E_ARG
            assert lib.get_option(opt) == hi
        assert lib._L.spcn_set_option(4, 0) == lib.SPCN_E_ARG
        assert lib.get_option(4) == -1 and lib.get_option(-1) == -1
    finally:
        for o, v in enumerate(saved):
            lib.set_option(o, v)


@pytest.mark.parametrize("kw,frag", [
    (dict(n=0), "n_samples"),
    (dict(n=(1 << 20) + 1), "n_samples"),
    (dict(white=0), "white_sum"),
    (dict(white=766), "white_sum"),
    (dict(q=0.0), "percentile"),
    (dict(q=100.5), "percentile"),
    (dict(out=None), "i0_out is NULL"),
    (dict(wsn=16), "workspace"),
])
def test_estimate_i0_rejects(lib, kw, frag):
    a = dict(n=1000, white=660, q=80.0, out=C.c_void_p(1 << 24), wsn=1 << 26)
    a.update(kw)
    st = lib._L.spcn_estimate_i0(C.c_void_p(1 << 20), 16, 16, a["n"], C.c_uint64(1), a["white"], a["q"], a["out"],
                                 None, C.c_void_p(1 << 28), a["wsn"], None)
    assert st in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
    assert frag in lib._L.spcn_last_error().decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(n=0), "n_samples"),
    (dict(n=262145), "n_samples"),
    (dict(lam=float("nan")), "lambda_nmf"),
    (dict(lam=-0.5), "lambda_nmf"),
    (dict(it=-1), "n_iter"),
    (dict(wsn=16), "workspace"),
])
def test_estimate_basis_rejects(lib, kw, frag):
    """Host-side validation of the basis fit's arguments: nothing is enqueued."""
    a = dict(n=200000, lam=0.1, it=50, wsn=1 << 30)
    a.update(kw)
    p = lib.params()
    st = lib._L.spcn_estimate_basis(C.c_void_p(1 << 20), 64, 64, C.byref(p), C.c_float(a["lam"]), a["n"], C.c_uint64(1),
                                    a["it"], None, C.c_void_p(1 << 24), None, None, None, C.c_void_p(1 << 28),
                                    a["wsn"], None)
    assert st in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
    assert frag in lib._L.spcn_last_error().decode()


def test_estimate_i0_workspace_size(lib):
    assert lib.workspace_size(lib.OP_ESTIMATE_I0, 0, 0, 100000) > 100000 * 8
    assert lib.workspace_size(lib.OP_ESTIMATE_I0, 0, 0, (1 << 20) + 1) == 0


def test_streamed_rejects(lib):
    p = lib.params()
    ok = dict(src=C.c_void_p(1 << 20), out=C.c_void_p(2 << 20), h=64, w=64, rows=16, wsn=1 << 26,
              comp=C.c_void_p(0), cin=C.c_void_p(8), cout=C.c_void_p(8))
    def call(**kw):
        a = dict(ok); a.update(kw)
        return lib._L.spcn_normalize_streamed(a["src"], a["out"], a["h"], a["w"], C.c_void_p(1 << 24),
                                              C.c_void_p(1 << 24), C.c_void_p(1 << 24), None, C.byref(p), a["rows"],
                                              None, C.c_void_p(1 << 28), a["wsn"], a["comp"], a["cin"], a["cout"])
    for kw, frag in ((dict(src=None), "host_src"), (dict(rows=0), "chunk_rows"), (dict(wsn=64), "workspace"),
                     (dict(cin=C.c_void_p(0)), "copy streams"), (dict(h=0), "height"),
                     (dict(out=C.c_void_p((1 << 20) + 4)), "overlap")):
        assert call(**kw) in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
        assert frag in lib._L.spcn_last_error().decode(), (kw, lib._L.spcn_last_error())


def test_exact_percentile_rejects(lib):
    """Argument checks of spcn_exact_percentile run on the host before any launch."""
    p = lib.params()
    need = lib.workspace_size(lib.OP_EXACT_PERCENTILE, 0, 0, 0)
    assert need >= 2 * (1 << 24) * 8
    img, w, out, ws = C.c_void_p(1 << 20), C.c_void_p(1 << 24), C.c_void_p(1 << 25), C.c_void_p(1 << 28)
    for args, frag in (((None, 8, 8, w, C.byref(p), out, None, ws, need, None), "img is NULL"),
                       ((img, 8, 8, None, C.byref(p), out, None, ws, need, None), "w is NULL"),
                       ((img, 8, 8, w, C.byref(p), None, None, ws, need, None), "p99_out is NULL"),
                       ((img, 0, 8, w, C.byref(p), out, None, ws, need, None), "height and width"),
                       ((img, 8, 8, w, C.byref(p), out, None, ws, need - 1, None), "workspace"),
                       ((img, 8, 8, w, C.byref(p), out, None, None, need, None), "workspace")):
        st = lib._L.spcn_exact_percentile(*args)
        assert st in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
        assert frag in lib._L.spcn_last_error().decode()


def test_recolor_p99_rejects(lib):
    p = lib.params()
    src, w, sc, P = C.c_void_p(1 << 20), C.c_void_p(1 << 24), C.c_void_p(1 << 25), C.c_void_p(1 << 26)
    def call(out, io=None):
        return lib._L.spcn_recolor_p99(src, 16, 16, w, w, sc, io, C.byref(p), P, out, None, None, None)
    assert call(C.c_void_p((1 << 20) + 12)) == lib.SPCN_E_ARG
    assert "overlap" in lib._L.spcn_last_error().decode()
    assert call(C.c_void_p(1 << 22), (C.c_float * 3)(255.0, -1.0, 255.0)) == lib.SPCN_E_ARG
    assert "i0_out" in lib._L.spcn_last_error().decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(mode=4), "mode"),
    (dict(mode=-1), "mode"),
    (dict(src=None), "src is NULL"),
    (dict(dst=None), "dst is NULL"),
    (dict(n=15), "multiple of 16"),
    (dict(src=C.c_void_p((1 << 20) + 8)), "aligned"),
    (dict(dst=C.c_void_p((1 << 20) + 64)), "overlap"),
    (dict(mode=1, ws=None), "workspace"),
    (dict(mode=3, ws=None), "workspace"),
    (dict(mode=2, dst=None), "dst is NULL"),
])
def test_bandwidth_probe_rejects(lib, kw, frag):
    args = dict(src=C.c_void_p(1 << 20), dst=C.c_void_p(1 << 24), n=1 << 12, mode=0, ws=C.c_void_p(1 << 26),
                wsn=1 << 22)
    args.update(kw)
    st = lib._L.spcn_bandwidth_probe(args["src"], args["dst"], args["n"], args["mode"], args["ws"], args["wsn"], None)
    assert st in (lib.SPCN_E_ARG, lib.SPCN_E_WORKSPACE)
    assert frag in lib._L.spcn_last_error().decode()
