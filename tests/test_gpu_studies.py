"""The one-GPU parameter studies (partitioning scheme, overlap) on small grids:
every case converges in both modes, the communication volume equals the
oracle's, the synchronous sweep counts equal the oracle's, and more overlap
never needs more synchronous sweeps on these Laplace problems (Sec. 4.3)."""
import sys

import numpy as np
import pytest

import ras_inputs as R
from oracle import overlap as oover
from oracle import partition as opart
from oracle import schwarz

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_owner(A, scheme, P):
    if scheme == "regular_1d":
        return opart.regular_1d(A.n, P)
    if scheme == "regular_2d":
        # the most nearly square factorisation P = px * py, px >= py
        px, py = min(((P // d, d) for d in range(1, P + 1) if P % d == 0 and P // d >= d),
                     key=lambda f: f[0] - f[1])
        return opart.regular_grid(A.grid, (px, py))
    return opart.rcb(A.coords(), P, 0, 0.0)


def _oracle_sweeps(A, owner, gamma, tol):
    b = R.uniform_rhs(A.n, 1)
    _, _, k = schwarz.RAS(A, owner, gamma, "chol", "fp64").sync(b, tol, 5000)
    return k


def _check_rows(rows):
    for r in rows:
        A = R.laplace2d(r["grid"])
        owner = _oracle_owner(A, r["partitioner"], r["parts"])
        vol = oover.comm_volume(owner, oover.subdomain_sets(A, owner, r["overlap"]))
        assert r["comm"]["total_values"] == int(vol.sum()), r
        assert r["comm"]["max_neighbours"] == int(np.count_nonzero(vol, axis=1).max()), r
        assert r["sync"]["converged"] and r["async"]["converged"], r
        assert r["sync"]["rel_residual"] < 1e-8 and r["async"]["rel_residual"] < 1e-8, r
        k = _oracle_sweeps(A, owner, r["overlap"], 1e-8)
        assert abs(r["sync"]["sweeps"] - k) <= 1, (r["sync"]["sweeps"], k, r)


def test_overlap_study_small():
    from paper_2003_05361_amd import studies

    _say("overlap study: 40^2, 4 parts, overlaps 0,1,2,4")
    rows = studies.main(["overlap", "--sizes", "40", "--overlaps", "0,1,2,4", "--nparts", "4",
                         "--max-seconds", "20"])
    assert [r["overlap"] for r in rows] == [0, 1, 2, 4]
    _check_rows(rows)
    sweeps = [r["sync"]["sweeps"] for r in rows]
    assert all(a >= b for a, b in zip(sweeps, sweeps[1:])), sweeps
    vols = [r["comm"]["total_values"] for r in rows]
    assert all(a < b for a, b in zip(vols, vols[1:])), vols


def test_partitioner_study_small():
    from paper_2003_05361_amd import studies

    _say("partitioner study: 4 parts of 256 unknowns, overlap 2")
    rows = studies.main(["partitioners", "--parts", "4", "--per-part", "256", "--overlap", "2",
                         "--max-seconds", "20"])
    assert [r["partitioner"] for r in rows] == ["regular_1d", "regular_2d", "rcb"]
    _check_rows(rows)
    # strips have at most two neighbours (Sec. 3.2.1)
    assert rows[0]["comm"]["max_neighbours"] <= 2
    assert rows[0]["sync_speedup_vs_1d"] == 1.0


@pytest.mark.parametrize("loc,k", [("chol", 0), ("cg", 8)])
def test_phase_breakdown_accounts_for_the_kernel_time(loc, k):
    """The measured per-phase times (residual, local solve, prolongation, other) of
    each subdomain's workgroup add up to its share of the kernel time."""
    import torch

    import paper_2003_05361_amd as ras

    _say(f"case: phase breakdown {loc}")
    A = R.laplace2d(96)
    b = torch.tensor(R.uniform_rhs(A.n, 3), dtype=torch.float64, device="cuda")
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local(loc, "fp64", k))
    _, info = h.solve(b, tol=0.0, mode="sync", max_sweeps=200, team=1 if loc == "cg" else 0)
    ph = h.phase_seconds()
    ks = info[0]["kernel_seconds"]
    assert ph.shape == (16, 4) and np.all(ph >= 0)
    per_wg = ph.sum(axis=1)  # one subdomain per workgroup here
    assert np.all(per_wg <= 1.02 * ks) and np.all(per_wg >= 0.7 * ks), (per_wg, ks)
    assert np.all(ph[:, 1] > 0) and np.all(ph[:, 0] > 0)
    _, info = h.solve(b, tol=1e-8, mode="async", max_sweeps=100000, max_seconds=30, team=1 if loc == "cg" else 0)
    ph = h.phase_seconds()
    assert np.all(ph >= 0) and np.all(ph.sum(axis=1) <= 1.02 * info[0]["kernel_seconds"])
    h.close()
