"""CPU runs under AddressSanitizer + UndefinedBehaviorSanitizer (any report fails the run): the FP64
oracle built with gcc's sanitizers runs its pin tests, and the C-ABI host layer (argument checks,
workspace sizes, error strings) built with clang's host-side sanitizers runs the ABI tests.  Each
run is a subprocess with the sanitizer runtime preloaded; it must report the instrumented library
as the one it loaded."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load(path, name):
    import importlib.util
    spec = importlib.util.spec_from_file_location(name, os.path.join(ROOT, path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(env_extra, tests, marker):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    # the first test module prints which libraries the process mapped, so the run proves what it ran
    probe = ("import os;m=open('/proc/self/maps').read();"
             f"print('{marker}', 'asan' in m, os.environ.get('SPCN_ORACLE_LIB') or os.environ.get('SPCN_LIB'))")
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0 and f"{marker} True" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", *tests], env=env,
                       capture_output=True, text=True, cwd=ROOT, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    ob = _load("oracle/build.py", "_oracle_build_san")
    lib = ob.build(out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    out = _run({"SPCN_ORACLE_LIB": lib, "LD_PRELOAD": asan},
               ["tests/test_oracle_solve.py", "tests/test_oracle_percentile.py", "tests/test_oracle_modes.py",
                "tests/test_oracle_i0.py", "tests/test_oracle_nmf_grad.py"], "oracle-asan")
    print(out.strip().splitlines()[-1])


def test_abi_host_layer_under_asan_ubsan(tmp_path):
    sb = _load("paper_1901_03088_amd/build.py", "_spcn_build_san")
    try:
        rt = sb.sanitizer_runtime()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    lib = sb.build_sanitized(str(tmp_path / "libspcn_asan.so"))
    out = _run({"SPCN_LIB": lib, "LD_PRELOAD": rt}, ["tests/test_abi.py"], "abi-asan")
    print(out.strip().splitlines()[-1])
