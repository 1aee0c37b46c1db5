"""Build ``libtetrt.so`` (the C-ABI library) for gfx950 with hipcc, in-tree;
and ``libtetrt_probe.so``, the benchmark's L1 calibration kernel, which is not
part of the traversal library."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtetrt.so")
PROBE_LIB = os.path.join(HERE, "libtetrt_probe.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("api.cpp", "batch.cpp", "server.cpp", "pack.cpp", "walk.hip",
                                                    "sort.hip", "serve.hip", "noalloc.hip")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("pack.h", "device.h", "handle.h")] + [
    os.path.join(ROOT, "include", "tetrt.h")]
PROBE_SOURCES = [os.path.join(HERE, "csrc", "probe_l1.hip")]

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-pthread",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(out: str, sources, deps, force: bool, verbose: bool) -> str:
    if not force and os.path.exists(out):
        newest = max(os.path.getmtime(p) for p in list(sources) + list(deps))
        if os.path.getmtime(out) >= newest:
            return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp] + list(sources)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, out)
    return out


def build_library(force: bool = True, verbose: bool = False) -> str:
    """Compile the traversal library; with ``force=False`` only when a source is newer."""
    return _compile(LIB, SOURCES, HEADERS, force, verbose)


def build_probe(force: bool = True, verbose: bool = False) -> str:
    """Compile the benchmark's calibration library (libtetrt_probe.so)."""
    return _compile(PROBE_LIB, PROBE_SOURCES, [], force, verbose)


if __name__ == "__main__":
    print(build_library(force=True))
    print(build_probe(force=True))
