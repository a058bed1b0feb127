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


def test_traffic_hash_covers_every_kernel_source():
    import glob
    import os
    csrc = os.path.join(bench.ROOT, "paper_1401_5245_amd", "csrc")
    found = {os.path.relpath(p, bench.ROOT) for p in glob.glob(os.path.join(csrc, "*"))}
    assert set(bench.KERNEL_SOURCES) == found
    assert "paper_1401_5245_amd/csrc/edge_grey.hip" in bench.KERNEL_SOURCES


def test_host_cores_bounded():
    assert 1 <= bench.host_cores() <= 16


def _fake_detail():
    rl = {"bound": "hbm", "achieved": 4700.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.5875,
          "traffic": None}
    return {
        "plain_512": {"us_per_launch": 2.0, "gpx_s": 131.0, "bit_exact": True},
        "plain_8192": {"us_per_launch": 5.39, "gpx_s": 12450.0, "roofline": rl, "bit_exact": True},
        "plain_65536": {"gpx_s": 23255.0, "roofline": rl, "sampled_rows_bit_exact": True},
        "full_65536": {"full": {"gpx_s": 23000.0, "roofline": rl, "sampled_rows_bit_exact": True},
                       "full_vs_plain_time": 1.01},
        "batched_4096": {"gpx_s_graph_of_20": 4400.0,
                         "speedup_graph_of_20_vs_per_image_graph": 860.0,
                         "bit_exact_all_crops": True},
        "serving": {"p99_bound_ms": 20.0, "speedup_at_p99_bound": 16.4,
                    "batched": {"max_sustained": {"gpx_s": 249.2, "p50_ms": 0.68,
                                                  "p99_ms": 1.08}}},
    }


def test_final_line_is_compact_and_complete():
    import json
    args = bench.parse(["--steps", "20", "--warmup", "5"])
    head = {"ms_per_step": 0.0142, "bytes_per_step": 2 * 16384 * 256 * 8,
            "pixels_per_step": 16384 ** 2, "warmup_launches": 1400,
            "trials_ms": [0.0142 + 1e-5 * k for k in range(10)],
            "cfg": {"vec_words": 4, "rows_per_tile": 32, "waves_per_block": 4,
                    "blocks_per_cu": 1, "cache_policy": 2},
            "bit_exact_full": True, "bit_exact_clause2": True, "replays_equal": True}
    cpu = {"value": 0.64, "unit": "Gpixel/s", "cores": 1, "kind": "oracle",
           "sample": "28 x the 16384x16384 headline image, full definition, byte image in and "
                     "out (packing excluded), 12.1 s on one thread of AMD EPYC 9575F 64-Core "
                     "Processor"}
    line = bench.compact_line(head, args, 67832099, cpu, bench.summarise(_fake_detail()),
                              os.path.join(bench.ROOT, "gpurun_out", "bench_detail.json"))
    text = json.dumps(line)
    assert len(text) < 2048, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in line, k
    assert line["steps"] == 20 and line["n_gpus"] == 1
    assert set(line["roofline"]) == {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert abs(line["roofline"]["frac"] - line["roofline"]["achieved"] / 8000.0) < 1e-4
    # value and achieved describe the same per-step time
    gbs = line["value"] * 1e9 * 0.25 / 1e9
    assert abs(gbs - line["roofline"]["achieved"]) / gbs < 0.01
    assert "model" not in line["config"] and "workload" in line["config"]
    assert set(line["others"]) == {"cfg1_plain_512_u32", "cfg2_plain_8192_u64", "plain_65536_u64",
                                   "full_65536_u64", "cfg3_batched_4096_u32", "cfg5_served_u64"}


def test_sustained_rate_stops_at_the_first_failure():
    runs = [{"offered_rps": r, "p99_ms": p} for r, p in
            ((1e4, 1.0), (2e4, 2.0), (4e4, 30.0), (8e4, 3.0), (1.6e5, 40.0))]
    best, later = bench.sustained(runs, 20.0)
    assert best["offered_rps"] == 2e4
    assert later == [8e4]
    best, later = bench.sustained(runs[:2], 20.0)
    assert best["offered_rps"] == 2e4 and later == []
    best, later = bench.sustained([{"offered_rps": 1, "p99_ms": 99.0}], 20.0)
    assert best is None and later == []
