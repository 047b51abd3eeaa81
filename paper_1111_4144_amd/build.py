"""Build libcholinv.so (the gfx950 HIP kernels + the C-ABI of include/cholinv.h).

    python -m paper_1111_4144_amd.build [-j JOBS] [-v]

Every source under csrc/ is compiled by hipcc for gfx950 into _build/, then
linked into paper_1111_4144_amd/libcholinv.so (in-tree, so the library ships
with the source tree).  Packed FP32 instructions are disabled for the device
code (-packed-fp32-ops); the compiler still emits ordinary FP32/FP64 FMAs.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcholinv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CXXFLAGS = [
    "-x", "hip", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-I" + INCLUDE, "-I" + CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-pragma-unroll-threshold=1000000",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-warning-option",
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _deps(path, seen=None):
    """The source and every local header it includes (recursively)."""
    import re
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path) as f:
        for inc in re.findall(r'#include\s+"([^"]+)"', f.read()):
            for d in (CSRC, INCLUDE):
                q = os.path.join(d, inc)
                if os.path.exists(q):
                    _deps(q, seen)
    return seen


def _compile(src, verbose, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(d) for d in _deps(src)):
        return obj
    cmd = [HIPCC, *CXXFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stdout))
    if verbose and out.strip():
        print(out, flush=True)
    return obj


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental=True skips objects newer than their
    inputs; the default always recompiles) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    # the longest translation units first, so they do not finish last
    srcs = sorted(srcs, key=lambda p: -os.path.getsize(p) if p.endswith(".hip") else 0)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def source_digest() -> str:
    """Digest of every kernel source and header (ties measured counters to code)."""
    h = hashlib.sha256()
    for s in _sources() + sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + \
            [os.path.join(INCLUDE, "cholinv.h")]:
        with open(s, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args()
    print(build(a.j, a.v, a.incremental))
    sys.exit(0)
