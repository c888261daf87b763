"""Build libtpasym.so (HIP for gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel (the exact tier is slow to
compile), then linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtpasym.so")

SOURCES = ["tp_pass.hip", "tp_exact.hip", "tp_energy.hip", "tp_noalloc.hip", "tp_host.cpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # every fused multiply-add is written explicitly: the error bounds count roundings
    "-ffp-contract=off", "-fno-fast-math",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


# Per-source flags.  The energy kernels keep their MFMA accumulators in the
# VGPR form: with accumulation registers the compiler copies every tile out of
# them once per loop iteration.
SOURCE_FLAGS = {"tp_energy.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(name, path, extra, verbose):
    obj = os.path.join(OBJ, os.path.basename(path) + ".o")
    cmd = [_hipcc(), *FLAGS, *SOURCE_FLAGS.get(name, []), *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
           path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {path}:\n{r.stdout}{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False, extra=(), sources=None, out=None) -> str:
    """Compile every source (or ``sources``: {name: path}) and link ``out`` (default libtpasym.so)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = {s: os.path.join(CSRC, s) for s in SOURCES}
    srcs.update(sources or {})
    with ThreadPoolExecutor(len(srcs)) as ex:
        res = list(ex.map(lambda kv: _compile(kv[0], kv[1], list(extra), verbose), srcs.items()))
    for _, err in res:
        if verbose and err.strip():
            sys.stderr.write(err)
    lib = out or LIB
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in res], "-o", lib + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv,
                extra=["-Rpass-analysis=kernel-resource-usage"] if "-r" in sys.argv else ()))
