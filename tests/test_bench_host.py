"""Host-side parts of bench.py that run without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_the_oracle_on_a_bounded_sample():
    import bench
    from paper_1712_01294_amd import workloads as W
    w = W.jittered_sine(n_side=12)
    out = bench.cpu_baseline(w, 0.5)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "pairs/s"
    assert out["value"] > 0.0
    assert "targets" in out["sample"]


def test_algorithmic_units_and_fingerprint():
    import bench
    n, G, F, P = 1000, 20000, 30000, 15000
    b, f = bench.algorithmic("hydro_fluxes", n, G, F, P)
    assert b == 288.0 * n + 4.0 * F and f == 236.0 * P
    b, f = bench.algorithmic("hydro_fluxes_mfv", n, G, F, P)
    assert b == 296.0 * n + 4.0 * F and f == 310.0 * P
    fp = bench.source_fingerprint()
    assert len(fp) == 16 and int(fp, 16) >= 0
    for (wl, k), v in bench.TRAFFIC.items():
        assert v["bytes_per_launch"] > 0 and len(v["fingerprint"]) == 16
