"""Host-side pieces of the parameter studies (no GPU): the communication
summary, the square split of the 2-D scheme and the markdown summary."""
import numpy as np

from paper_2003_05361_amd import studies


def test_square_split():
    assert studies._square_split(16) == (4, 4)
    assert studies._square_split(6) == (3, 2)
    assert studies._square_split(7) == (7, 1)


def test_comm_summary():
    vol = np.array([[0, 3, 0], [3, 0, 2], [0, 2, 0]], dtype=np.int64)
    s = studies.comm_summary(vol)
    assert s["total_values"] == 10 and s["max_recv"] == 5 and s["max_neighbours"] == 2
    assert abs(s["mean_neighbours"] - 4 / 3) < 1e-15


def test_markdown_summary():
    row = {"grid": 64, "parts": 4, "partitioner": "rcb", "overlap": 2, "max_band": 40, "band_entries": 1000,
           "comm": {"total_values": 10, "max_neighbours": 2},
           "sync": {"converged": True, "sweeps": 30, "seconds": 0.01, "ms_per_sweep": 0.33},
           "async": {"converged": False, "seconds": 0.02, "local_solves_median": 41.0},
           "async_free": {"converged": True, "seconds": 0.03, "local_solves_median": 52.0},
           "async_speedup": 0.5, "async_free_speedup": 0.33,
           "measured_share_sync": {"residual": 0.2, "local_solve": 0.6, "prolong": 0.1, "other": 0.1},
           "measured_share_async": {"residual": 0.25, "local_solve": 0.55, "prolong": 0.1, "other": 0.1}}
    md = studies.markdown("overlap", [row], {"overlap 2": np.eye(2, dtype=np.int64)}, "python -m x overlap")
    assert "| 64^2 | 4 | rcb | 2 | 40 |" in md
    assert "0.0200 (41 not conv.)" in md and "0.0300 (52)" in md
    assert "| 0 | 1 | . |" in md
    assert "| 0.20 / 0.60 / 0.10 / 0.10 | 0.25 / 0.55 / 0.10 / 0.10 |" in md


def test_time_to_tolerance_summary():
    rows = [{"config": "c", "n": 16, "local": "chol-fp64", "mode": "sync", "converged": True, "seconds": 10.0, "sweeps": 100,
             "ms_per_sweep": 100.0, "local_solves_min": 100, "local_solves_median": 100.0, "local_solves_max": 100,
             "rel_residual": 9e-9, "rel_residual_host_plain": 9e-9},
            {"config": "c", "n": 16, "local": "chol-fp64", "mode": "async", "converged": True, "seconds": 8.0,
             "local_solves_min": 90, "local_solves_median": 95.0, "local_solves_max": 99, "rel_residual": 8e-9, "rel_residual_host_plain": 8e-9}]
    md = studies.markdown_ttt(rows, "python -m x time_to_tolerance")
    assert "| chol-fp64 | sync | True | 10.0 | 100 | 100.000 | 100 / 100 / 100 | 9.000e-09 | 9.000e-09 | - |" in md
    assert "| chol-fp64 | async | True | 8.0 | - | - | 90 / 95 / 99 | 8.000e-09 | 8.000e-09 | - |" in md
    assert "speedup over synchronous: 1.250" in md


def test_byte_model_parts():
    from paper_2003_05361_amd.perfmodel import local_solve_parts

    # n = 10 local rows, 8 owned, K = 5, w = 3, nnz(L) = 20
    res, loc, pro = local_solve_parts([10, 8, 5, 3, 20], "chol_sparse", "fp64", 0)
    assert res == 10 * (12 * 5 + 16) and pro == 8 * (16 + 8)
    assert loc == 2 * ((20 + 10) * (8 + 4) + 16 * 10) + 2 * 10 * 8
    _, loc_b, _ = local_solve_parts([10, 8, 5, 3], "chol", "fp16", 0)
    assert loc_b == 2 * 10 * 4 * 2 + 4 * 10 * 4 + 2 * 10 * 4
    _, loc_c, _ = local_solve_parts([10, 8, 5, 3], "cg", "fp32", 8)
    assert loc_c == 8 * 10 * (5 * 8 + 11 * 4)


def test_batching_summary():
    rows = [{"mode": "sync", "systems": 4, "rhs": 9, "unknowns": 1000, "one_launch_per_system_s": 2.0,
             "one_batched_launch_s": 0.5, "speedup": 4.0, "all_converged": True}]
    md = studies.markdown_batching(rows, "python -m x batching")
    assert "| sync | 4 | 9 | 1000 | 2.000 | 0.500 | 4.00 | True |" in md


def test_oras_summary():
    rows = [{"config": "c", "n": 16, "local": "chol-fp64", "tol": 1e-8, "robin_q": 1.0,
             "sync": {"converged": True, "seconds": 1.0, "sweeps": 100},
             "async": {"converged": True, "seconds": 0.8, "local_solves_median": 90.0}},
            {"config": "c", "n": 16, "local": "chol-fp64", "tol": 1e-8, "robin_q": 0.3,
             "sync": {"converged": True, "seconds": 0.5, "sweeps": 40},
             "async": {"converged": False, "seconds": 0.4, "local_solves_median": 45.0}}]
    md = studies.markdown_oras(rows, "python -m x oras")
    assert "| 0.3 | 40 | 0.500 | 0.400 (45 not conv.) | 2.50x fewer |" in md
