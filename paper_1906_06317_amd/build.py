"""Builds libppa.so for gfx950 with hipcc (in-tree, next to this file).

Each HIP source is compiled to an object in parallel, then the objects are
linked into one shared library.  build() always recompiles every source;
build(incremental=True) recompiles only sources older than their object or
than any header of the library.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(HERE, "..", "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libppa.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code; the compiler
# otherwise forms them from ordinary float code.
FLAGS = [
    "--offload-arch=gfx950", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(INCLUDE, "*.h"))


def _obj(src):
    return os.path.join(OBJ, os.path.splitext(os.path.basename(src))[0] + ".o")


def _stale(src, newest_header):
    o = _obj(src)
    if not os.path.exists(o):
        return True
    t = os.path.getmtime(o)
    return t < os.path.getmtime(src) or t < newest_header


def _compile(src, verbose):
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-c", "-o", _obj(src) + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(_obj(src) + ".tmp", _obj(src))


def build(verbose: bool = False, incremental: bool = False, jobs: int | None = None) -> str:
    """Compile the HIP sources and link libppa.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    newest = max((os.path.getmtime(h) for h in _headers()), default=0.0)
    todo = [s for s in srcs if not incremental or _stale(s, newest)]
    jobs = jobs or min(16, max(1, os.cpu_count() or 1), max(1, len(todo)))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, s, verbose) for s in todo]:
            f.result()
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
               *[_obj(s) for s in srcs]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
