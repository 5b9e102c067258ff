"""Build libdm.so (the HIP kernels and the C ABI of include/dm.h) for gfx950.

Usage: python -m paper_2210_15114_amd.build   (or paper_2210_15114_amd.build.build())

Every .hip file under csrc/ is compiled to an object with hipcc, then linked
into paper_2210_15114_amd/libdm.so.  Packed FP32 instructions are disabled
(-packed-fp32-ops) for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdm.so")
ROOT = os.path.dirname(HERE)

ARCH = os.environ.get("DM_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + CSRC,
    "-I" + os.path.join(ROOT, "include"),
]


# Per-file code generation options.  The sort-free FP64 matrix-core kernels
# keep their accumulators in ordinary VGPRs: with the default choice the
# compiler copied the accumulators between VGPRs and AGPRs around every
# product step (v_accvgpr_read/write), which took the b = 64 moments kernels
# from about 0.17 to 0.26 ms.  (The same option made the low-rank update
# kernel several times slower, so it applies to this file only.)
FILE_FLAGS = {
    "k_sortfree.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + CFLAGS + FILE_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)


def code_hash(paths) -> str:
    """First 16 hex digits of the sha256 of the given source files with their
    comments removed and whitespace runs collapsed: figures stored beside the
    sources (counter traffic, sampled errors) name the code they were taken
    with, and stay valid across edits of comments only."""
    h = hashlib.sha256()
    for p in paths:
        t = open(p, encoding="utf-8").read()
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(re.sub(r"\s+", " ", t).strip().encode())
        h.update(b"\0")
    return h.hexdigest()[:16]
