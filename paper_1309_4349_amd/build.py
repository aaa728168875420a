"""Build libkk.so (the HIP kernels and the C ABI) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkk.so")
SOURCES = ["kk_sweep.hip", "kk_aux.hip", "kk_tri.hip", "kk_api.cpp", "kk_batch.cpp", "kk_tri_batch.cpp", "kk_serve.cpp",
           "kk_noalloc.hip", "kk_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = [ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln]
    return r.returncode, errs


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link libkk.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="kkbuild") as d:
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[HIPCC, *FLAGS, "-c", "-o", o, s] for s, o in zip(srcs, objs)]
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            results = list(ex.map(lambda c: _run(c, verbose), cmds))
        errs = [ln for _, e in results for ln in e]
        if any(rc != 0 for rc, _ in results):
            sys.stderr.write("\n".join(errs) + "\n")
            raise RuntimeError("hipcc failed building libkk.so")
        rc, lerrs = _run([HIPCC, *FLAGS, "-shared", "-o", tmp, *objs], verbose)
        errs += lerrs
        if rc != 0:
            sys.stderr.write("\n".join(errs) + "\n")
            raise RuntimeError("hipcc failed linking libkk.so")
    if verbose and errs:
        print("\n".join(errs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
