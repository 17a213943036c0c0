"""Build the gfx950 shared library ``librtc.so`` in-tree with hipcc.

Usage: ``python -m paper_1903_01852_amd.build``.  Always recompiles: each
source to an object in ``_build/`` (in parallel), then one link.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "librtc.so")
OBJ = os.path.join(PKG, "_build")
SOURCES = ["rtc_kernels.hip", "rtc_persist.hip", "rtc_engine.cpp", "rtc_serve.cpp",
           "rtc_pacer.cpp"]
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]
NOISE = "packed-fp32-ops"     # the host pass does not know this target feature


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [ln for ln in (res.stdout + res.stderr).splitlines() if NOISE not in ln]
    return res.returncode, msgs


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        jobs.append((obj, [cc, *HIP_FLAGS, "-c", f"-I{INCLUDE}", f"-I{CSRC}",
                           os.path.join(CSRC, src), "-o", obj]))
    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
        results = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    for (obj, _), (rc, msgs) in zip(jobs, results):
        if rc != 0:
            raise RuntimeError(f"hipcc failed for {os.path.basename(obj)}:\n" + "\n".join(msgs))
        if verbose and msgs:
            print("\n".join(msgs))
    out_tmp = LIB + ".tmp"
    rc, msgs = _run([cc, *HIP_FLAGS, "-shared", *[o for o, _ in jobs], "-o", out_tmp,
                     "-lpthread"], verbose)
    if rc != 0:
        raise RuntimeError("link failed:\n" + "\n".join(msgs))
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
