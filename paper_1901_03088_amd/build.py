"""Builds libspcn.so (HIP, gfx950) in-tree with hipcc: one object per source, then one link."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspcn.so")
ARCH = "gfx950"
# Packed FP32 instructions are switched off for every HIP source (they are not used by design).
HIPFLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = ["hipcc", *HIPFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer for the C-ABI layer (argument checks,
# workspace carving, error reporting): each flag applies to the host compilation only; device code
# is built as usual.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_sanitized(out: str, verbose: bool = False) -> str:
    """A copy of libspcn.so at `out` whose host code in spcn_api.hip is instrumented (the other
    objects come from the regular build); load it with the clang ASan runtime preloaded
    (sanitizer_runtime())."""
    if not all(os.path.exists(os.path.join(OBJ, os.path.basename(s) + ".o"))
               for s in glob.glob(os.path.join(CSRC, "*.hip"))):
        build(verbose)
    api = os.path.join(CSRC, "spcn_api.hip")
    obj = out + ".api.o"
    cmd = ["hipcc", *HIPFLAGS, *HOST_SANITIZE, "-c", api, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {api}:\n{r.stderr}")
    others = [os.path.join(OBJ, os.path.basename(s) + ".o") for s in sorted(glob.glob(os.path.join(CSRC, "*.hip")))
              if os.path.basename(s) != "spcn_api.hip"]
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out, obj, *others,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return out


def sanitizer_runtime() -> str:
    """Path of the clang ASan runtime the instrumented library needs preloaded."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
