"""Build libpts.so (and the issue-rate probe libpts_probe.so) for gfx950 with hipcc.

Usage: ``python -m paper_2607_16946_amd.build``.  Objects go to ``_build/``
(not committed); the shared libraries are written next to this file, where
the binding loads them.  Packed FP32 instructions are disabled for all device
code (``-target-feature -packed-fp32-ops``).
"""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("PTS_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function"] + DEVICE_FLAGS

LIB = os.path.join(PKG, "libpts.so")
PROBE_LIB = os.path.join(PKG, "libpts_probe.so")


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if "warning" in warn:
        print(warn, file=sys.stderr)


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed for {out}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(jobs: int = 8) -> list[str]:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    probe_srcs = sorted(glob.glob(os.path.join(CSRC, "probe", "*.hip")))
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    pobjs = [os.path.join(BUILD, "probe_" + os.path.basename(s) + ".o") for s in probe_srcs]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o) for s, o in zip(srcs + probe_srcs, objs + pobjs)]
        for f in futs:
            f.result()
    _link(objs, LIB)
    _link(pobjs, PROBE_LIB)
    return [LIB, PROBE_LIB]


if __name__ == "__main__":
    for p in build():
        print(p)
