"""Builds libps.so (the gfx950 HIP library) in-tree with hipcc.

Every translation unit is compiled for gfx950 only, with packed FP32
arithmetic disabled in the device code generator.  Object files go to
``paper_1003_4322_amd/_build``; the library lands next to this file.

The library carries the hash of the sources and flags it was built from
(``ps_build_hash``); the binding refuses to load a library whose hash differs
from the sources in the tree, so a stale build can never be the one tested.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HEADER = os.path.join(ROOT, "include", "ps.h")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libps.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [f"k_{p}_{t}.hip" for p in ("zcurl", "zepi", "xpass", "strided") for t in ("f32", "f64")] + [
    "k_spectrum.hip", "ps_api.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def src_hash() -> str:
    """SHA-256 (first 16 hex digits) of every file the library is built from
    (csrc/*, include/ps.h, this file's source list and flags), byte for byte."""
    h = hashlib.sha256()
    h.update(repr((SOURCES, FLAGS)).encode())
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp", ".h")))
    for f in files:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    with open(HEADER, "rb") as fh:
        h.update(b"ps.h")
        h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, defs) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build(jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    defs = [f'-DPS_SRC_HASH="{src_hash()}"']
    # the longest translation units first, so that they do not finish last
    order = sorted(SOURCES, key=lambda s: ("xpass" not in s, "zepi" not in s, s))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, defs), order))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 0))
