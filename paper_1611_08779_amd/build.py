"""Builds libocd.so (HIP, gfx950) in-tree: ``python paper_1611_08779_amd/build.py``
(run as a script: importing the package would load the library being built).

Every translation unit under ``csrc/`` is compiled with hipcc for gfx950 only,
with packed-FP32 instruction selection switched off, and linked into
``paper_1611_08779_amd/libocd.so``.  Objects go to ``_build/`` at the repo root.
"""

from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(ROOT, "_build", "ocd")
LIB = os.path.join(PKG, "libocd.so")

SOURCES = ["ocd_api.hip", "ocd_forward.hip", "ocd_forward_reg.hip", "ocd_backward.hip", "ocd_train.hip",
           "ocd_jobs.hip",
           "ocd_mmse.hip", "ocd_fixed.hip", "ocd_ofdm.hip", "ocd_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    noise = ("packed-fp32-ops", "not a recognized feature")
    warn = "\n".join(l for l in r.stderr.splitlines() if l and not any(n in l for n in noise))
    if warn.strip():
        print(warn, file=sys.stderr)
    return obj


def build(jobs: int | None = None) -> str:
    """Compiles every source and links ``libocd.so``; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
