"""Build libedgemask.so (HIP, gfx950) in-tree with hipcc.

The library is several HIP translation units (the edge kernels and the C
ABI; the grey-input kernels; the peeling kernels in four ranges of level
counts), compiled in parallel and linked into one shared object.

This module imports nothing from the package, so it can be loaded by its
path before the library exists.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HEADER = os.path.join(ROOT, "include", "edge_masks.h")
LIB = os.path.join(HERE, "libedgemask.so")
ARCH = "gfx950"


def units() -> list:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def deps() -> list:
    return units() + sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [HEADER, __file__]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c",
            # no packed-FP32 instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-o", obj, src]


def link_command(objs: list, out: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs


def _run(cmd: list) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile the library; always recompiles. Returns the .so path."""
    srcs = units()
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory(prefix="edgemask_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s)[:-4] + ".o") for s in srcs]
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda so: _run(compile_command(*so)), zip(srcs, objs)))
        tmp = LIB + ".tmp"
        _run(link_command(objs, tmp))
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} units")
    return LIB


def is_stale() -> bool:
    """True when the library is missing or older than any source it is
    built from."""
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in deps())


if __name__ == "__main__":
    print(build(verbose=True))
