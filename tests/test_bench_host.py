"""Host-side parts of bench.py that run without a GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_the_oracle_on_a_bounded_sample():
    """A whole-set oracle pass over the median sub-cube of the set, single-
    threaded and on the OpenMP build, with the host's CPU model."""
    import bench
    from paper_1712_01294_amd import workloads as W
    w = W.clustered(n_side=40, seed=W.SEED_BASE + 150)
    subs = bench.cpu_sample(w)
    assert len(subs) == 4 and len({p for _, p in subs}) == 4
    ns = [sub.n for sub, _ in subs]
    assert ns == sorted(ns) and 0 < ns[0] and ns[-1] < w.n
    for sub, _ in subs:
        assert sub.periodic == (0, 0, 0)
        assert np.all((sub.x >= 0) & (sub.x < 0.125)) and np.all((sub.z >= 0) & (sub.z < 0.125))
    one, omp = bench.cpu_baseline(w)
    assert one["kind"] == "oracle" and one["cores"] == 1 and one["unit"] == "pairs/s"
    assert omp["kind"] == "oracle_omp" and omp["cores"] >= 1
    assert one["value"] > 0.0 and omp["value"] > 0.0
    assert "sub-cube" in one["sample"] and one["cpu_model"]


def test_algorithmic_units_and_fingerprint():
    import bench
    n, G, F, P = 1000, 20000, 30000, 15000
    assert bench.algorithmic("solve_h", n, G, F, P, 5.0) == (48.0 * n, 20.0 * G * 5.0, 4.0 * G)
    assert bench.algorithmic("gradients", n, G, F, P) == (264.0 * n, 65.0 * G, 4.0 * F)
    assert bench.algorithmic("hydro_fluxes", n, G, F, P) == (288.0 * n, 400.0 * P, 4.0 * F)
    assert bench.algorithmic("hydro_fluxes_mfv", n, G, F, P) == (296.0 * n, 475.0 * P, 4.0 * F)
    assert bench.binding(0.01, 0.02) == "alu" and bench.binding(0.02, 0.01) == "hbm"
    fp = bench.source_fingerprint()
    assert len(fp) == 16 and int(fp, 16) >= 0
    for table in (bench.TRAFFIC, bench.COUNTERS):
        for (wl, k), v in table.items():
            assert len(v["fingerprint"]) == 16


def test_recorded_counters_belong_to_the_current_kernel_sources():
    """The traffic and VALU tables were taken on the kernel sources as they
    stand (the bench reports them as null otherwise)."""
    import bench
    fp = bench.source_fingerprint()
    for table in (bench.TRAFFIC, bench.COUNTERS):
        assert table and all(v["fingerprint"] == fp for v in table.values())
