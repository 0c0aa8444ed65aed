"""Build libtnrsvd.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1707_07803_amd.build  (or call build()).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtnrsvd.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["kernels_contract.hip", "kernels_sweep.hip", "kernels_wide.hip", "kernels_grad.hip",
           "kernels_adjoint.hip", "kernels_sparse.hip", "kernels_round.hip", "tnrsvd_abi.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are disabled for every kernel of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libtnrsvd.so next to this file."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    # -z defs: a symbol no object defines fails the link, not the first load
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized(outdir: str, verbose: bool = False) -> str:
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer on
    its HOST code (device code is not instrumented), for host-only tests of the
    argument checks.  Rebuilt only when a source changed; returns the path."""
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES + ["tnrsvd_internal.h", "wg_linalg.h"]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "tnrsvd.h"), "rb").read())
    tag = h.hexdigest()[:16]
    os.makedirs(outdir, exist_ok=True)
    lib = os.path.join(outdir, f"libtnrsvd_san_{tag}.so")
    if os.path.exists(lib):
        return lib
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + [
        "-O1", "-g", "-fno-omit-frame-pointer",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def comp(src):
        obj = os.path.join(outdir, os.path.splitext(src)[0] + f"_{tag}.o")
        r = subprocess.run([hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(comp, SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
