"""Builds libmhd_ens.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: python -m paper_2108_05110_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmhd_ens.so")
SOURCES = ["mesh.cpp", "tiling.cpp", "assemble.hip", "solve.hip", "adjoint.hip", "capi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for the device code (the compiler still
# vectorises ordinary float arithmetic into other instructions).  hipcc hands
# -Xclang options to the host pass as well, which reports the target feature as
# unknown for x86; that one warning is dropped from the build log.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
_HOST_FEATURE_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    lines = [ln for ln in p.stdout.splitlines() if _HOST_FEATURE_NOTE not in ln]
    if lines:
        print("\n".join(lines), flush=True)
    if p.returncode != 0:
        raise subprocess.CalledProcessError(p.returncode, cmd)


def build(verbose: bool = False, jobs: int = 0) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = DEVICE_FLAGS
        else:
            cmd[1:1] = ["-x", "c++"]
        cmds.append(cmd)
        objs.append(obj)
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 1) // 2), 6)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = OUT + ".tmp"
    _run([HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
