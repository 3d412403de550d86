"""Build libnubulb.so (the stepper) and libnubulb_testhooks.so (its arithmetic primitives,
for tests) in-tree with hipcc for gfx950.

Flags: -ffp-contract=off keeps the arithmetic specification (no implicit fma);
-packed-fp32-ops is disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnubulb.so")
SOURCES = ["nb_kernels.hip", "nb_adjoint.hip", "nb_api.hip"]
HOOKS_LIB = os.path.join(HERE, "libnubulb_testhooks.so")
HOOKS_SOURCES = ["nb_testhooks.hip"]
ARCH = os.environ.get("NB_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def _compile(src: str, bdir: str, verbose: bool) -> str:
    obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    noise = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if verbose and noise:
        print("\n".join(noise))
    return obj


def _link(lib: str, objs: list, verbose: bool) -> None:
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = SOURCES + HOOKS_SOURCES
    with ThreadPoolExecutor(len(srcs)) as ex:
        objs = dict(zip(srcs, ex.map(lambda s: _compile(s, bdir, verbose), srcs)))
    _link(LIB, [objs[s] for s in SOURCES], verbose)
    _link(HOOKS_LIB, [objs[s] for s in HOOKS_SOURCES], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
