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
