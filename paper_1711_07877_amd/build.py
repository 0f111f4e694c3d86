"""Build the SBD shared library (libsbd.so) in-tree for gfx950.

HIP sources go through hipcc (--offload-arch=gfx950, packed-FP32 instructions
disabled); host-only C++ goes through g++.  Objects land in ``_build/`` next
to this file; the library in the package directory.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsbd.so")

HIP_SOURCES = ["fft.hip", "colconv.hip", "colconv_f32a.hip", "colconv_f32b.hip", "colconv_f32c.hip", "colconv_f64.hip",
               "rows.hip", "rows_f32.hip", "rows_f64.hip", "kernels.hip", "pairdiff.hip", "gmres.hip", "sbd_api.cpp"]
HOST_SOURCES = ["host/bessel.cpp", "host/sbd_fit.cpp", "host/layout.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Rpass-analysis=kernel-resource-usage"]
RESOURCES = os.path.join(BUILD, "kernel_resources.txt")
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-mavx2", "-mfma"]


def source_hash() -> str:
    """Short SHA-256 over every library source (used to tie stored counter data to a build)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "**", "*"), recursive=True)):
        if os.path.isfile(p) and p.endswith((".hip", ".cpp", ".h")):
            with open(p, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src.replace("/", "_") + ".o")
    if src in HIP_SOURCES:
        cmd = [HIPCC, *HIP_FLAGS, "-x", "hip", "-c", path, "-o", obj]
    else:
        cmd = ["g++", *HOST_FLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if src in HIP_SOURCES:
        with open(obj + ".resources.txt", "w") as fh:
            fh.write("\n".join(ln for ln in r.stderr.splitlines() if "kernel-resource-usage" in ln))
    return obj


def kernel_resources() -> dict:
    """{kernel symbol: {"VGPRs": int, "ScratchSize": int, "VGPRs Spill": int, ...}} from the
    compiler's resource-usage remarks of the last build."""
    import glob
    import re
    out, cur = {}, None
    for path in sorted(glob.glob(os.path.join(BUILD, "*.resources.txt"))):
        with open(path) as fh:
            for ln in fh:
                m = re.search(r"remark:\s+Function Name: (\S+)", ln)
                if m:
                    cur = out.setdefault(m.group(1), {})
                    continue
                m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[bytes/lane\])?: (\d+) \[", ln)
                if m and cur is not None:
                    cur[m.group(1).strip()] = int(m.group(2))
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link libsbd.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = HIP_SOURCES + HOST_SOURCES
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:  # fft.hip first: the longest
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
