"""Build the cmlb HIP library (libcmlb.so) for gfx950 with hipcc.

Usage: ``python -m paper_1808_04406_amd.build``.  The library is built
in-tree next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcmlb.so")
SOURCES = ["step_tp.hip", "step_tp2.hip", "step_d37.hip", "step2_d37.hip", "kernels.hip", "kernels_closure.hip", "api.cpp"]
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # no packed-FP32 instructions: scalar FP32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    """Compile every source to an object file (in parallel, in a temporary
    directory next to the library) and link the shared library."""
    import shutil
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmpdir = tempfile.mkdtemp(prefix=".build_", dir=HERE)
    try:
        objs, cmds = [], []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([hipcc] + FLAGS + ["-x", "hip", "-c", src, "-o", obj])
        workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
        with ThreadPoolExecutor(workers) as pool:
            for cmd, rc in zip(cmds, pool.map(lambda c: subprocess.call(c), cmds)):
                if verbose:
                    print(" ".join(cmd), flush=True)
                if rc:
                    raise subprocess.CalledProcessError(rc, cmd)
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
