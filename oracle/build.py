"""Build the FP64 CPU oracle (test infrastructure only) as oracle/liboracle.so with gcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    """Builds the oracle library at `out`; with sanitize, instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (any report aborts)."""
    src = os.path.join(HERE, "spcn_oracle.c")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", *san, "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
