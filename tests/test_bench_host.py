"""Host-side logic of the benchmark (no GPU): algorithmic byte counts, the
source-hash guard on measured traffic, and the refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_tile_bytes_packed():
    n = 4000
    # packed: 6 distinct entries per symmetric 3 x 3 block, N(N+1)/2 pairs
    assert bench.tile_bytes(n, "f64") == 6 * (n * (n + 1) // 2) * 8 == 384_096_000
    assert bench.tile_bytes(n, "f32") == 384_096_000 // 2
    assert bench.tile_bytes(n, "bf16") == 384_096_000 // 4


def test_ritz_extremes_of_an_exact_lanczos_run():
    """Lanczos on a diagonal matrix with a known spectrum, run in numpy with
    full reorthogonalisation: the extreme Ritz values converge to the extreme
    eigenvalues and their residual bounds bracket the error."""
    np = pytest.importorskip("numpy")
    rng = np.random.default_rng(3)
    lam = np.sort(np.concatenate([[0.05, 41.0], rng.uniform(0.3, 30.0, 398)]))
    q = rng.standard_normal(lam.size)
    q /= np.linalg.norm(q)
    Q = [q]
    alpha, beta = [], []
    qprev, bprev = np.zeros_like(q), 0.0
    for _ in range(120):
        w = lam * Q[-1] - bprev * qprev
        a = float(Q[-1] @ w)
        w -= a * Q[-1]
        for v in Q:
            w -= (v @ w) * v
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        qprev, bprev = Q[-1], b
        Q.append(w / b)
    tmin, tmax, rmin, rmax = bench.ritz_extremes(alpha, beta)
    assert abs(tmax - 41.0) <= max(rmax, 1e-9 * 41.0)
    assert abs(tmin - 0.05) <= max(rmin, 1e-9)
    assert abs(tmax - 41.0) < 1e-6 and abs(tmin - 0.05) < 1e-3


def test_power_fit_recovers_a_power_law():
    ns = [100, 200, 400, 1000, 2000, 4000]
    p, a = bench.power_fit(ns, [8.0 * n ** 0.6 for n in ns])
    assert abs(p - 0.6) < 1e-12 and abs(a - 8.0) < 1e-9


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
