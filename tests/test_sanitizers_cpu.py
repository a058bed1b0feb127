"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C functions run on every shape up to 9 x 9 and long thin ones
with exact-size heap buffers; the library's host code (argument checks of
every entry point, the host planner's table checks) is rebuilt with the
sanitizers on the host side only and driven by a C program with fake device
pointers that no call dereferences. Either program aborts on the first
report."""
import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "c_abi")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(HERE, "oracle_san.c"), os.path.join(ROOT, "oracle", "edge_oracle.c"),
                    "-o", exe], check=True)
    res = subprocess.run([exe], capture_output=True, text=True, env=SAN_ENV)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "oracle ok" in res.stdout


def _clang_rt_dir():
    hits = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux",
                                  "libclang_rt.asan-x86_64.so"))
    return os.path.dirname(hits[0]) if hits else None


def test_abi_validation_under_asan_and_ubsan(tmp_path):
    from paper_1401_5245_amd import build as hip_build
    rt = _clang_rt_dir()
    if rt is None:
        pytest.skip("the ROCm clang sanitizer runtime is not installed")
    san = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
                 "-fno-omit-frame-pointer", "-g"):
        san += ["-Xarch_host", flag]
    objs = []

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src)[:-4] + ".o"))
        res = subprocess.run(hip_build.compile_command(src, obj) + san, capture_output=True,
                             text=True)
        assert res.returncode == 0, res.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, hip_build.units()))
    lib = str(tmp_path / "libedgemask_san.so")
    subprocess.run([hip_build.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-shared-libasan", "-o", lib] + objs,
                   check=True)
    exe = str(tmp_path / "validate_san")
    subprocess.run([os.path.join(ROCM, "llvm", "bin", "clang"), "-std=c99", "-g",
                    "-fsanitize=address,undefined", "-shared-libasan",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "validate_san.c"), "-o", exe, "-L", str(tmp_path),
                    "-ledgemask_san", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
                    "-Wl,-rpath," + rt], check=True)
    # the HIP runtime's own allocations are not this library's: no leak report
    env = dict(SAN_ENV, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0")
    res = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    assert "validate ok" in res.stdout
