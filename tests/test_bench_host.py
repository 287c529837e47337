"""Host-side logic of the benchmark (no GPU): algorithmic byte counts, the
source-hash guard on measured traffic, and the refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_tile_bytes_packed_and_half():
    n = 4000
    # packed: 6 distinct entries per symmetric 3 x 3 block, N(N+1)/2 pairs
    assert bench.tile_bytes(n, "f64") == 6 * (n * (n + 1) // 2) * 8 == 384_096_000
    assert bench.tile_bytes(n, "f32") == 384_096_000 // 2
    assert bench.tile_bytes(n, "bf16") == 384_096_000 // 4
    # symmetric half of the 3N x 3N matrix
    assert bench.tile_bytes(n, "f64", packed=False) == 12000 * 12001 // 2 * 8


def test_traffic_is_null_for_other_sources():
    t = dict(bench.TRAFFIC)
    t["src_sha256"] = "0" * 64
    assert bench.measured_traffic(t) is None
    tb = dict(bench.TRAFFIC_BLOCK)
    tb["src_sha256"] = "0" * 64
    assert bench.measured_traffic(tb, "f32") is None


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_host_description_keys():
    h = bench.host_description()
    assert set(h) == {"cpu", "logical_cpus", "usable_cpus", "omp_num_threads"}
    assert h["logical_cpus"] >= 1
