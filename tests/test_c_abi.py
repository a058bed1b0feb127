"""The boundary is a plain C ABI: the header compiles as strict C99, and a
C program with no Python or PyTorch drives the library (device memory from
the HIP runtime's C API) and matches the oracle pixel for pixel."""
import os
import subprocess

import pytest

import oracle
from paper_1401_5245_amd import build as hip_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "c_abi")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_header_is_strict_c99():
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                    "-fsyntax-only", "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "header_c99.c")], check=True)


def build_c_program() -> str:
    """Compile run_edge.c against the library and the oracle (host code only)."""
    if not os.path.exists(hip_build.LIB):
        pytest.fail("libedgemask.so is not built")
    oracle._load()
    exe = os.path.join(HERE, "run_edge")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "run_edge.c"), "-o", exe,
           "-L", os.path.dirname(hip_build.LIB), "-ledgemask",
           "-L", os.path.join(ROOT, "oracle"), "-loracle",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.dirname(hip_build.LIB),
           "-Wl,-rpath," + os.path.join(ROOT, "oracle"), "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return exe


def test_c_program_builds():
    assert os.access(build_c_program(), os.X_OK)


@pytest.mark.gpu
def test_c_program_matches_oracle():
    exe = build_c_program()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "all match: 43 cases" in r.stdout
