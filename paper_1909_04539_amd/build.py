"""Build libsbs.so (the C-ABI solver library) for gfx950 with hipcc, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsbs.so")

# every source of the library: the HIP kernels (*.hip) and the host code (*.cpp)
SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU forms.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-pthread",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every source to an object file (in parallel), then link the
    shared library; the objects go to a temporary folder outside the tree."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with tempfile.TemporaryDirectory(prefix="sbs_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc(), *HIP_FLAGS, *(extra or []), "-I", INCLUDE, "-I", CSRC, "-c", s, "-o", o]
                for s, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for f in [ex.submit(subprocess.check_call, c) for c in cmds]:
                f.result()
        tmp = out + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
