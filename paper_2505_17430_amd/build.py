"""Build ``libsevo.so`` (the C-ABI library) from the HIP sources in ``csrc/``.

Every translation unit is compiled by hipcc for gfx950 only, then linked into
one shared library next to this file.  Usage: ``python -m
paper_2505_17430_amd.build [--incremental]``.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsevo.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-pass-failed",
    # packed FP32 instructions stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _inputs_digest(src: str) -> str:
    """Digest of what an object is compiled from: the flags, the source and
    every header.  It is read before the compiler starts, so an object whose
    inputs change while it compiles is recompiled by the next build."""
    hs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
    hs.append(os.path.join(os.path.dirname(HERE), "include", "sevo.h"))
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for path in [src, *hs]:
        with open(path, "rb") as f:
            h.update(path.encode() + b"\0" + f.read())
    return h.hexdigest()


def _compile(src: str, incremental: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    stamp = obj + ".inputs"
    digest = _inputs_digest(src)
    if incremental and os.path.exists(obj) and os.path.exists(stamp):
        with open(stamp) as f:
            if f.read().strip() == digest:
                return obj
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    with open(stamp, "w") as f:
        f.write(digest + "\n")
    return obj


def build(incremental: bool = False, jobs: int | None = None) -> str:
    """Compile and link libsevo.so; returns its path.  Raises on any error."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
