"""bench.py's host-side helpers (no GPU): occupancy summary, counter-traffic
lookup keyed by the kernel-source hash, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_occupancy_summary():
    occ = np.array([[0.0, 1, 5, 100], [0.5, 3, 2, 300], [1.0, 2, 0, 200], [2.0, 0, 0, 0]])
    s = bench.occupancy_summary(occ, 1000)
    assert s["active_max"] == 3 and s["queued_max"] == 5
    assert abs(s["active_mean"] - 2.0) < 1e-12  # (1*0.5 + 3*0.5 + 2*1.0) / 2
    assert abs(s["in_use_frac_of_budget_max"] - 0.3) < 1e-12
    assert len(s["active_timeline_10_bins"]) == 10
    assert bench.occupancy_summary(np.zeros((1, 4)), 10) is None


def test_traffic_lookup_follows_kernel_hash():
    path = os.path.join(ROOT, "profiles", "traffic_poisson2d_1024_8x8.json")
    t = json.load(open(path))
    ratio = t["counter_bytes_per_dispatch"] / t["algorithmic_bytes_per_dispatch"]
    got, src = bench.traffic_from_profiles("poisson2d_1024_8x8", 1000.0)
    if t["kernel_hash"] == bench.kernel_source_hash():
        assert abs(got - 1000.0 * ratio) < 1e-9 and src.startswith("derived_from_profile")
    else:
        assert got is None and src is None
    assert bench.traffic_from_profiles("no_such_workload", 1.0) == (None, None)


def test_host_cpu_is_stated():
    c = bench.host_cpu()
    assert c["os_cpu_count"] == os.cpu_count() and c["affinity"] >= 1


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in p.stderr


def test_resident_roofline_reports_the_counter_rate():
    """A cache-resident workload's roofline never reports the streaming-model rate
    as an HBM rate: achieved and frac come from the counters, or are null."""
    import bench

    roof = {"bound": "hbm", "achieved": 8740.0, "frac": 1.0925, "peak": 8000.0}
    bench.resident_roofline(roof, 4500.04)
    assert roof["achieved"] == 4500.0 and roof["frac"] == round(4500.04 / 8000.0, 4)
    assert roof["model_GBps"] == 8740.0
    roof = {"bound": "hbm", "achieved": 8740.0, "frac": 1.0925, "peak": 8000.0}
    bench.resident_roofline(roof, None)
    assert roof["achieved"] is None and roof["frac"] is None and roof["model_GBps"] == 8740.0
