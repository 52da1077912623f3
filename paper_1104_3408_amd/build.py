"""Build libshellspec.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled to an object file in parallel (the translation units
share no device code: each holds its own kernels and host launchers), then
the objects are linked into the shared library.

Usage: python -m paper_1104_3408_amd.build   (or call build()).
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libshellspec.so")

SOURCES = ["api.hip", "derivs.hip", "rhs.hip", "filter.hip", "bf16x3.hip", "noalloc.hip", "host_math.cpp",
           "tuning.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose=False, jobs=None):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    with tempfile.TemporaryDirectory(prefix="shellspec_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[hipcc] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with ThreadPoolExecutor(jobs) as ex:
            rcs = list(ex.map(lambda c: _run(c, verbose), cmds))
        if any(rcs):
            raise RuntimeError("hipcc failed compiling libshellspec sources")
        if _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", LIB + ".tmp"], verbose):
            raise RuntimeError("hipcc failed linking libshellspec.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
