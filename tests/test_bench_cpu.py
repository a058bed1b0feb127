"""Host-side pieces of bench.py: the refusal of more than one GPU, the
banded multi-thread run of the oracle used for the all-cores CPU figure,
and the traffic field that is dropped once the kernel sources change."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


@pytest.mark.parametrize("shape", [(1, 5), (2, 7), (5, 3), (17, 33), (100, 64)])
@pytest.mark.parametrize("threads", [1, 3, 8, 16])
@pytest.mark.parametrize("clauses", [1, 2, 3])
def test_banded_oracle_equals_whole_image(shape, threads, clauses):
    rng = np.random.default_rng(hash((shape, threads, clauses)) % 2**32)
    img = (rng.random(shape) < 0.6).astype(np.uint8)
    np.testing.assert_array_equal(bench.oracle_banded(img, threads, clauses),
                                  oracle.edge(img, clauses=clauses))


def test_traffic_requires_matching_source_hash(tmp_path):
    p = tmp_path / "profile.md"
    p.write_text("traffic_bytes_per_launch: 123\nkernel_source_sha256_16: 0000000000000000\n")
    assert bench.measured_traffic(str(p)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None


def test_traffic_takes_the_indexed_table(tmp_path):
    import hashlib
    import os
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(bench.ROOT, f), "rb") as fh:
            h.update(fh.read())
    cur = h.hexdigest()[:16]
    p = tmp_path / "two.md"
    p.write_text(f"# two kernels\ntraffic_bytes_per_launch: 111\nkernel_source_sha256_16: {cur}\n"
                 f"text: with a colon\ntraffic_bytes_per_launch: 222\n"
                 f"kernel_source_sha256_16: 0123456789abcdef\n")
    assert bench.measured_traffic(str(p)) == 111
    assert bench.measured_traffic(str(p), 0) == 111
    assert bench.measured_traffic(str(p), 1) is None        # taken with other sources
    assert bench.measured_traffic(str(p), 2) is None        # no third table


def test_host_cores_bounded():
    assert 1 <= bench.host_cores() <= 16
