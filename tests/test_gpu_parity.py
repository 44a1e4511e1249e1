"""GPU parity: the HIP path through the C ABI against the oracle (needs an MI355X).

Tolerances: float64 local solves -- the same iteration up to rounding order,
so histories agree to 1e-9 relative per sweep plus an absolute 1e-13 (the
relative residual of an iterate near convergence is itself computed with
about 1e-16 ||A|| ||x|| / ||b|| of cancellation error), iterates to 1e-9
relative; float32 local arithmetic -- iterates after a
fixed number of sweeps to 2e-5 relative (float32 unit roundoff 6e-8 times the
growth of CG / triangular-solve rounding over a few sweeps); converged
solutions to the acceptance criteria: relative residual below tol (exact,
recomputed) and 1e-6 relative error against the float64 direct solve where the
right-hand side makes that attainable.
"""
import sys

import numpy as np
import pytest

import ras_inputs as R
from oracle import partition as opart
from oracle import schwarz

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _ras():
    import paper_2003_05361_amd as ras

    ras.lib()
    return ras


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cuda(v):
    torch = _torch()
    return torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")


def _owner(A, kind, arg):
    if kind == "regular_1d":
        return opart.regular_1d(A.n, arg)
    if kind in ("regular_2d", "regular_3d"):
        return opart.regular_grid(A.grid, arg)
    P, seed, jit = arg
    return opart.rcb(A.coords(), P, seed, jit)


def _spec(ras, A, kind, arg):
    if kind == "rcb":
        P, seed, jit = arg
        return ras.partition("rcb", P, grid=A.grid, seed=seed, jitter=jit)
    return ras.partition(kind, arg, grid=A.grid)


def _oracle(A, kind, arg, gamma, loc, storage="fp64", k=0):
    return schwarz.RAS(A, _owner(A, kind, arg), gamma, loc, storage, k)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _agree(a, b, tol, what=""):
    """Iterate parity, normwise and element by element:
    ||a - b||_2 <= tol ||b||_2 and max_i |a_i - b_i| <= tol ||b||_inf."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    nrm = _rel(a, b)
    ew = float(np.max(np.abs(a - b), initial=0.0) / max(np.max(np.abs(b), initial=0.0), 1e-300))
    assert nrm <= tol and ew <= tol, (what, "normwise", nrm, "elementwise", ew, "tol", tol)


# ----------------------------------------------------------------------------- synchronous parity
def test_config1_sync_exact_history_and_solution():
    """64^2 Poisson, 4 strips, overlap 2, banded Cholesky FP64, sync to 1e-10."""
    ras = _ras()
    _say("case: poisson2d_64_strips4 sync chol fp64")
    A, b, cfg = R.config_problem("poisson2d_64_strips4")
    orc = _oracle(A, "regular_1d", 4, 2, "chol")
    xo, ho, ko = orc.sync(b, 1e-10, 10000)
    h = ras.setup(A, _spec(ras, A, "regular_1d", 4), 2, ras.local("chol", "fp64"))
    x, info = h.solve(_cuda(b), tol=1e-10, mode="sync", max_sweeps=10000)
    x = x.cpu().numpy()
    _, hg = h.residual_history()
    assert info[0]["converged"] and info[0]["sweeps"] == ko
    assert len(hg) == len(ho)
    assert np.all(np.abs(hg - ho) <= 1e-9 * ho + 1e-13)
    _agree(x, xo, 1e-9)
    assert info[0]["rel_residual"] < 1e-10
    xd = schwarz.direct_solve(A, b)
    assert _rel(x, xd) <= 1e-6
    assert _rel(x, cfg["x_star"]) <= 1e-6
    assert np.all(h.local_solve_counts() == ko)


@pytest.mark.parametrize("N,part,gamma,k", [
    (48, ("regular_2d", (3, 3)), 2, 6),
    (37, ("regular_2d", (2, 3)), 1, 4),  # ragged boxes and tails
    (40, ("regular_1d", 5), 0, 3),  # zero overlap: block Jacobi with CG
])
def test_sync_cg_fp64_matches_oracle(N, part, gamma, k):
    ras = _ras()
    _say(f"case: sync cg fp64 N={N} part={part} gamma={gamma} k={k}")
    A = R.laplace2d(N, N + 3)
    b = R.uniform_rhs(A.n, 11)
    orc = _oracle(A, part[0], part[1], gamma, "cg", "fp64", k)
    h = ras.setup(A, _spec(ras, A, *part), gamma, ras.local("cg", "fp64", k))
    for sweeps in (1, 2, 7):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, info = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        assert info[0]["sweeps"] == sweeps
        _agree(x.cpu().numpy(), xo, 1e-9)
        _, hg = h.residual_history()
        assert np.all(np.abs(hg - ho) <= 1e-9 * ho + 1e-13)


@pytest.mark.parametrize("team", [1, 2, 4, 8, 16])
def test_sync_cg_team_sizes_match_oracle(team):
    """Several workgroups per subdomain (halo exchange + team reductions) give the
    same iteration as the oracle, for every team size."""
    ras = _ras()
    _say(f"case: sync cg fp64 team={team}")
    A = R.laplace2d(70, 61)
    b = R.uniform_rhs(A.n, 21)
    part = ("regular_2d", (2, 2))
    orc = _oracle(A, *part, 3, "cg", "fp64", 7)
    h = ras.setup(A, _spec(ras, A, *part), 3, ras.local("cg", "fp64", 7))
    for sweeps in (1, 4):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, info = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps, team=team)
        _agree(x.cpu().numpy(), xo, 1e-9)
        _, hg = h.residual_history()
        assert np.all(np.abs(hg - ho) <= 1e-9 * ho + 1e-13)
    xa, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=100000, max_seconds=60, team=team)
    assert info[0]["converged"] and schwarz.relative_residual(A, xa.cpu().numpy(), b) < 1e-8


@pytest.mark.parametrize("team", [1, 4])
def test_ordered_cg_team_is_multiplicative_schwarz(team):
    ras = _ras()
    _say(f"case: ordered cg team={team}")
    A = R.laplace2d(40)
    b = R.uniform_rhs(A.n, 15)
    part = ("regular_2d", (2, 3))
    orc = _oracle(A, *part, 2, "cg", "fp64", 5)
    h = ras.setup(A, _spec(ras, A, *part), 2, ras.local("cg", "fp64", 5))
    xo, _ = orc.ordered(b, 3)
    x, _ = h.solve(_cuda(b), tol=0.0, mode="ordered", max_sweeps=3, team=team)
    _agree(x.cpu().numpy(), xo, 1e-9)


def test_sync_cg_fp32_3d_rcb_matches_oracle():
    ras = _ras()
    _say("case: sync cg fp32 3d rcb")
    A = R.laplace3d(14)
    b = R.uniform_rhs(A.n, 12)
    part = ("rcb", (9, 3, 0.4))
    orc = _oracle(A, *part, 1, "cg", "fp32", 8)
    h = ras.setup(A, _spec(ras, A, *part), 1, ras.local("cg", "fp32", 8))
    for sweeps in (1, 4):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, 2e-5)
    # and it converges to the float64 tolerance (correction form)
    x, info = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=5000)
    assert info[0]["converged"] and info[0]["rel_residual"] < 1e-8


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-9), ("fp32", 2e-5), ("fp16", 2e-5)])
def test_sync_band_storage_matches_oracle(storage, tol):
    ras = _ras()
    _say(f"case: sync band {storage}")
    g = R.gaussian_random_field_2d(56, 8.0, 4)
    A = R.tpfa2d(np.exp(2.0 * g), 10.0)
    b = R.uniform_rhs(A.n, 5)
    part = ("regular_2d", (3, 2))
    orc = _oracle(A, *part, 3, "chol", storage)
    h = ras.setup(A, _spec(ras, A, *part), 3, ras.local("chol", storage))
    for sweeps in (1, 3):
        xo, _, _ = orc.sync(b, 0.0, sweeps)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, tol)
    x, info = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=20000)
    assert info[0]["converged"] and info[0]["rel_residual"] < 1e-8


# band widths around the slab kernel's block structure (32-row blocks): near
# columns partly outside the band (w < 63), far columns present, the widest slab
# band (<= 144), and the row-major pass (w > 144)
@pytest.mark.parametrize("case,storage,tol", [
    ("2d70_w36", "fp64", 1e-9), ("2d100_w52", "fp32", 2e-5), ("3d16_w97", "fp64", 1e-9),
    ("3d20_w141", "fp64", 1e-9), ("3d20_w141", "fp16", 2e-5), ("3d24_w193", "fp64", 1e-9), ("3d24_w193", "fp32", 2e-5)])
def test_sync_band_widths_match_oracle(case, storage, tol):
    ras = _ras()
    _say(f"case: band width {case} {storage}")
    A, part, gamma = {
        "2d70_w36": (R.laplace2d(70), ("regular_2d", (2, 1)), 1),
        "2d100_w52": (R.laplace2d(100), ("regular_2d", (2, 2)), 2),
        "3d16_w97": (R.laplace3d(16), ("regular_3d", (2, 2, 2)), 2),
        "3d20_w141": (R.laplace3d(20), ("regular_3d", (2, 2, 1)), 2),
        "3d24_w193": (R.laplace3d(24), ("regular_3d", (2, 2, 1)), 2),
    }[case]
    b = R.uniform_rhs(A.n, 21)
    orc = _oracle(A, *part, gamma, "chol", storage)
    h = ras.setup(A, _spec(ras, A, *part), gamma, ras.local("chol", storage))
    w_expect = int(case.split("_w")[1])
    assert h.stats()["max_band"] == w_expect
    for sweeps in (1, 2):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, tol)


# sparse Cholesky local solves (nested dissection, level-scheduled triangular
# passes): exact local solves like the band, so the synchronous iterates match the
# oracle's exact-solve RAS to rounding (float64) or float32 rounding growth
@pytest.mark.parametrize("case,storage,tol", [
    ("2d96_4x4_g3", "fp64", 1e-9), ("3d16_rcb6_g1", "fp64", 1e-9), ("2d_strips_w320", "fp64", 1e-9),
    ("2d96_4x4_g3", "fp32", 2e-5), ("3d16_rcb6_g1", "fp32", 2e-5)])
def test_sync_sparse_cholesky_matches_oracle(case, storage, tol):
    ras = _ras()
    _say(f"case: sparse cholesky {case} {storage}")
    A, part, gamma = {
        "2d96_4x4_g3": (R.laplace2d(96), ("regular_2d", (4, 4)), 3),
        "3d16_rcb6_g1": (R.laplace3d(16), ("rcb", (6, 5, 0.3)), 1),
        "2d_strips_w320": (R.laplace2d(320, 24), ("regular_1d", 2), 2),
    }[case]
    b = R.uniform_rhs(A.n, 22)
    orc = _oracle(A, *part, gamma, "chol", "fp64")
    h = ras.setup(A, _spec(ras, A, *part), gamma, ras.local("chol_sparse", storage))
    for sweeps in (1, 3):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, tol, (sweeps, _rel(x.cpu().numpy(), xo)))
    _, hist, _ = orc.sync(b, 0.0, 6)
    h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=6)
    _, hh = h.residual_history()
    if storage == "fp64":
        assert np.all(np.abs(hh[:7] - hist[:7]) <= 1e-9 * hist[:7] + 1e-13)


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_async_sparse_cholesky_converges(storage):
    """Asynchronous (paced and free-running) sparse local solves reach the tolerance,
    also where the natural-order band (grid width 700) is too wide for the band solver."""
    ras = _ras()
    for A, part, gamma in [(R.laplace2d(96), ("regular_2d", (4, 4)), 3),
                           (R.laplace2d(700, 20), ("regular_1d", 2), 2)]:
        _say(f"case: async sparse {A.grid} {part} {storage}")
        b = R.uniform_rhs(A.n, 23)
        xd = schwarz.direct_solve(A, b)
        h = ras.setup(A, _spec(ras, A, *part), gamma, ras.local("chol_sparse", storage))
        for pace in (None, 0.0):
            x, info = h.solve(_cuda(b), tol=1e-9, mode="async", max_sweeps=100000, max_seconds=60, pace=pace)
            xx = x.cpu().numpy()
            assert info[0]["converged"], info
            assert schwarz.relative_residual(A, xx, b) < 1e-9
            assert _rel(xx, xd) <= 1e-6


def test_async_banded_runs_converge_every_time():
    """Regression: asynchronous banded runs on many concurrent workgroups converge
    in every repeat, with a bounded number of local solves (every update works on
    one snapshot of the values it reads)."""
    ras = _ras()
    _say("case: async banded repeats")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 16)
    xd = schwarz.direct_solve(A, b)
    for st in ("fp64", "fp32"):
        h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local("chol", st))
        for rep in range(5):
            x, info = h.solve(_cuda(b), tol=1e-10, mode="async", max_sweeps=5000, max_seconds=60)
            xx = x.cpu().numpy()
            assert info[0]["converged"], info
            assert info[0]["max_local_solves"] < 2000, info
            assert schwarz.relative_residual(A, xx, b) < 1e-10
            assert _rel(xx, xd) <= 1e-8


def test_single_subdomain_is_direct_solve():
    ras = _ras()
    _say("case: one subdomain")
    A = R.laplace2d(30, 17)
    b = R.uniform_rhs(A.n, 13)
    h = ras.setup(A, ras.partition("regular_1d", 1), 0, ras.local("chol", "fp64"))
    x, info = h.solve(_cuda(b), tol=1e-12, mode="sync", max_sweeps=5)
    assert info[0]["sweeps"] == 1 and info[0]["converged"]
    _agree(x.cpu().numpy(), schwarz.direct_solve(A, b), 1e-12)


def test_tiny_and_ragged_subdomains():
    """Subdomains smaller than a block of the banded solve and than a wavefront."""
    ras = _ras()
    _say("case: tiny ragged")
    A = R.laplace2d(7, 5)
    b = R.uniform_rhs(A.n, 14)
    part = ("regular_1d", 6)
    # the sparse solver's subdomains here (11 to 20 rows) are single leaves or
    # nearly so: some keep no dense block at all, and one lane group covers a step
    for loc, st, k, oloc, tol in (("chol", "fp64", 0, "chol", 1e-9), ("cg", "fp64", 3, "cg", 1e-9),
                                  ("chol_sparse", "fp64", 0, "chol", 1e-9), ("chol_sparse", "fp32", 0, "chol", 2e-5)):
        _say(f"case: tiny ragged {loc} {st}")
        orc = _oracle(A, *part, 1, oloc, "fp64", k)
        h = ras.setup(A, _spec(ras, A, *part), 1, ras.local(loc, st, k))
        xo, _, _ = orc.sync(b, 0.0, 3)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=3)
        _agree(x.cpu().numpy(), xo, tol, (loc, st))
        h.close()


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_one_unknown_and_a_chain(mode):
    """Degenerate systems: one unknown (each local solve is one division) and a
    1-D chain of 16 unknowns in two overlapping halves; every local solver and
    storage reaches the direct solution, in both modes."""
    ras = _ras()
    one = R.CSR(np.array([0, 1], np.int64), np.array([0], np.int32), np.array([4.0]), (1, 1, 1))
    chain = R.laplace2d(16, 1)
    for A, P, gamma in ((one, 1, 0), (chain, 2, 1)):
        b = R.uniform_rhs(A.n, 41) + 0.5
        xd = schwarz.direct_solve(A, b)
        for loc, st, k in (("chol", "fp64", 0), ("chol", "fp32", 0), ("chol", "fp16", 0),
                           ("chol_sparse", "fp64", 0), ("chol_sparse", "fp32", 0),
                           ("cg", "fp64", 10), ("cg", "fp32", 10)):
            _say(f"case: degenerate n={A.n} P={P} {loc} {st} {mode}")
            h = ras.setup(A, ras.partition("regular_1d", P, grid=A.grid), gamma, ras.local(loc, st, k))
            x, info = h.solve(_cuda(b), tol=1e-12, mode=mode, max_sweeps=500, max_seconds=30)
            assert info[0]["converged"], (loc, st, info)
            _agree(x.cpu().numpy(), xd, 1e-9, (A.n, loc, st))
            h.close()


def test_point_subdomains_are_jacobi():
    """One grid point per subdomain and no overlap: every local matrix is the
    point's diagonal entry, a synchronous sweep is a Jacobi step,
    x <- x + D^-1 (b - A x), and an ordered pass a Gauss-Seidel sweep in point
    order, for every local solver."""
    ras = _ras()
    A = R.laplace2d(5, 4)
    S = A.scipy().tocsr()
    d = S.diagonal()
    b = R.uniform_rhs(A.n, 43)
    xs, x = [], np.zeros(A.n)
    gs, y = [], np.zeros(A.n)
    for _ in range(4):
        x = x + (b - S @ x) / d
        xs.append(x)
        y = y.copy()
        for i in range(A.n):
            y[i] += (b[i] - (S[i] @ y)[0]) / d[i]
        gs.append(y)
    for loc, st, k in (("chol", "fp64", 0), ("chol", "fp32", 0), ("chol_sparse", "fp64", 0), ("cg", "fp64", 2)):
        _say(f"case: point subdomains {loc} {st}")
        h = ras.setup(A, ras.partition("regular_1d", A.n, grid=A.grid), 0, ras.local(loc, st, k))
        tol = 1e-13 if st == "fp64" else 5e-7
        for sweeps in (1, 4):
            xg, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
            _agree(xg.cpu().numpy(), xs[sweeps - 1], tol, (loc, st, sweeps))
            xo, _ = h.solve(_cuda(b), tol=0.0, mode="ordered", max_sweeps=sweeps)
            _agree(xo.cpu().numpy(), gs[sweeps - 1], tol, ("ordered", loc, st, sweeps))
        h.close()


@pytest.mark.parametrize("N,storage", [(27, "fp64"), (34, "fp32")])
def test_sparse_cholesky_at_lds_capacity(N, storage):
    """One 3-D box with nearly as many rows as the sparse solve keeps in LDS
    (19,683 of 19,968 in FP64; 39,304 of 39,936 in FP32), overlap 0: one sweep
    from zero is the direct solve (FP64), and in FP32 the sweeps are iterative
    refinement with a single-precision factor, each gaining several digits.
    The right-hand side comes from a known solution, so no reference solve is
    needed."""
    ras = _ras()
    _say(f"case: sparse at LDS capacity {N}^3 {storage}")
    A = R.laplace3d(N)
    assert A.n <= ras.sparse_max_rows(storage) < A.n + 1024
    xs = R.uniform_rhs(A.n, 31)
    b = A.scipy() @ xs
    h = ras.setup(A, ras.partition("rcb", 1, grid=A.grid, seed=5, jitter=0.3), 0, ras.local("chol_sparse", storage))
    x, info = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=1)
    _agree(x.cpu().numpy(), xs, 1e-11 if storage == "fp64" else 1e-4, "one sweep")
    x, info = h.solve(_cuda(b), tol=1e-13, mode="sync", max_sweeps=8)
    assert info[0]["converged"] and info[0]["sweeps"] <= (1 if storage == "fp64" else 5), info
    _agree(x.cpu().numpy(), xs, 1e-10, "converged")
    h.close()


# ----------------------------------------------------------------------------- ordered = RMS
@pytest.mark.parametrize("loc,k", [("chol", 0), ("cg", 5), ("chol_sparse", 0)])
def test_ordered_mode_is_multiplicative_schwarz(loc, k):
    ras = _ras()
    _say(f"case: ordered {loc}")
    A = R.laplace2d(40)
    b = R.uniform_rhs(A.n, 15)
    part = ("regular_2d", (2, 3))
    # the sparse solver is exact like the band: the same multiplicative iterates
    orc = _oracle(A, *part, 2, "chol" if loc == "chol_sparse" else loc, "fp64", k)
    h = ras.setup(A, _spec(ras, A, *part), 2, ras.local(loc, "fp64", k))
    for passes in (1, 3):
        xo, _ = orc.ordered(b, passes)
        x, info = h.solve(_cuda(b), tol=0.0, mode="ordered", max_sweeps=passes)
        assert info[0]["min_local_solves"] == passes and info[0]["max_local_solves"] == passes
        _agree(x.cpu().numpy(), xo, 1e-9)


# ----------------------------------------------------------------------------- asynchronous
@pytest.mark.parametrize("loc,st,k", [("chol", "fp64", 0), ("cg", "fp64", 10), ("chol", "fp32", 0)])
def test_async_converges_and_verifies(loc, st, k):
    ras = _ras()
    _say(f"case: async {loc} {st}")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 16)
    xd = schwarz.direct_solve(A, b)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local(loc, st, k))
    for run in range(3):
        x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=200000, max_seconds=60)
        xx = x.cpu().numpy()
        assert info[0]["converged"], info
        assert schwarz.relative_residual(A, xx, b) < 1e-8
        assert _rel(xx, xd) <= 1e-6
        counts = h.local_solve_counts()
        assert counts.min() >= 1 and counts.sum() == info[0]["total_local_solves"]


@pytest.mark.parametrize("loc,k,detect", [("chol", 0, "central"), ("cg", 10, "decentral"),
                                           ("chol_sparse", 0, "estimate")])
def test_failed_verification_resumes(loc, k, detect):
    """A detector that tests 100 tol fires before the tolerance is reached; the
    exact verification that follows the stop fails, and the iteration resumes
    from the current iterate (Sec. 3.3.2) until a stop passes it: more than one
    launch, converged, verified residual below tol, the direct solution.  A
    synchronous solve ignores the factor (its stop is the exact residual)."""
    ras = _ras()
    _say(f"case: resume after failed verification {loc} {detect}")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 18)
    xd = schwarz.direct_solve(A, b)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local(loc, "fp64", k))
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", detect=detect, max_sweeps=200000, max_seconds=60,
                      detect_factor=100.0)
    xx = x.cpu().numpy()
    assert info[0]["converged"] and info[0]["launches"] >= 2, info
    assert schwarz.relative_residual(A, xx, b) < 1e-8
    assert _rel(xx, xd) <= 1e-6
    _, plain = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=100000)
    _, scaled = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=100000, detect_factor=100.0)
    assert scaled[0]["sweeps"] == plain[0]["sweeps"] and scaled[0]["converged"], (plain, scaled)
    h.close()


@pytest.mark.parametrize("loc,st,k,team", [("chol", "fp64", 0, 0), ("cg", "fp64", 10, 4), ("cg", "fp32", 6, 1),
                                            ("chol_sparse", "fp64", 0, 0)])
def test_async_decentralized_detection(loc, st, k, team):
    ras = _ras()
    _say(f"case: async decentral {loc} {st} team={team}")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 17)
    xd = schwarz.direct_solve(A, b)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local(loc, st, k))
    for run in range(2):
        x, info = h.solve(_cuda(b), tol=1e-8, mode="async", detect="decentral", max_sweeps=200000, max_seconds=60,
                          team=team)
        xx = x.cpu().numpy()
        assert info[0]["converged"], info
        assert schwarz.relative_residual(A, xx, b) < 1e-8
        assert _rel(xx, xd) <= 1e-6


@pytest.mark.parametrize("loc,st,k,team", [("chol", "fp64", 0, 0), ("chol_sparse", "fp32", 0, 0),
                                          ("cg", "fp64", 10, 4)])
def test_async_estimate_detection(loc, st, k, team):
    """The estimate detector (the library's option: stop on the owned-residual
    estimate once every subdomain has updated) still returns only verified
    solutions."""
    ras = _ras()
    _say(f"case: async estimate {loc} {st} team={team}")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 17)
    xd = schwarz.direct_solve(A, b)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local(loc, st, k))
    for run in range(2):
        x, info = h.solve(_cuda(b), tol=1e-8, mode="async", detect="estimate", max_sweeps=200000, max_seconds=60,
                          team=team)
        xx = x.cpu().numpy()
        assert info[0]["converged"], info
        assert schwarz.relative_residual(A, xx, b) < 1e-8
        assert _rel(xx, xd) <= 1e-6


@pytest.mark.parametrize("pace", [0.0, 0.25, 16.0])
def test_async_paced_reads(pace):
    """Paced reads wait for slower neighbours before reading (bounded by pace times
    the previous update's duration).  Evenly loaded banded subdomains then need
    about as many updates as synchronous sweeps; every pace converges to the
    direct solution."""
    ras = _ras()
    _say(f"case: async chol fp64 pace={pace}")
    A = R.laplace2d(128)
    b = R.uniform_rhs(A.n, 1)
    xd = schwarz.direct_solve(A, b)
    h = ras.setup(A, ras.partition("rcb", 6, grid=A.grid, seed=0, jitter=0.0), 4, ras.local("chol", "fp64"))
    _, si = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=100000, max_seconds=60)
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=200000, max_seconds=60, pace=pace)
    xx = x.cpu().numpy()
    assert info[0]["converged"], info
    assert schwarz.relative_residual(A, xx, b) < 1e-8
    assert _rel(xx, xd) <= 1e-6
    if pace > 0:
        assert np.median(h.local_solve_counts()) <= 1.15 * si[0]["sweeps"], (h.local_solve_counts(), si)


def test_async_paced_cg_teams_converge():
    ras = _ras()
    _say("case: async cg fp64 team=4 pace=0.5")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 18)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local("cg", "fp64", 10))
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=200000, max_seconds=60, team=4, pace=0.5)
    assert info[0]["converged"], info
    assert schwarz.relative_residual(A, x.cpu().numpy(), b) < 1e-8


def test_solve_options_out_of_range_are_argument_errors():
    ras = _ras()
    _say("case: solve option argument errors")
    A = R.laplace2d(16)
    b = _cuda(R.uniform_rhs(A.n, 1))
    h = ras.setup(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol", "fp64"))
    for bad in (16.5, float("nan")):
        with pytest.raises(ras.RasError) as e:
            h.solve(b, tol=1e-8, mode="async", pace=bad)
        assert e.value.status == -1
    for kw in (dict(tol=-1.0), dict(tol=float("nan")), dict(max_sweeps=0), dict(detect_factor=-1.0),
               dict(detect_factor=float("nan"))):
        with pytest.raises(ras.RasError) as e:
            h.solve(b, **{"tol": 1e-8, "mode": "sync", **kw})
        assert e.value.status == -1, kw
    # mode and detector codes outside the enums, through the C ABI itself
    import ctypes as C
    x = b.clone()
    info = (ras.SolveInfo * 1)()
    for mode, det in ((7, 0), (0, 9)):
        opts = ras.SolveOpts(mode, det, 1e-8, 100, 0.0, 0, 0, -1.0)
        st = ras.lib().ras_solve(h._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), 1, C.byref(opts), info)
        assert st == -1 and b"unknown" in ras.lib().ras_last_error(), (mode, det)
    _, info = h.solve(b, tol=1e-8, mode="async", max_seconds=30)
    assert info[0]["converged"]


# ----------------------------------------------------------------------------- multi-RHS and batching
@pytest.mark.parametrize("loc", [("cg", 6), ("chol_sparse", 0)])
def test_multi_rhs_equals_single_sync(loc):
    ras = _ras()
    _say(f"case: multi rhs {loc}")
    torch = _torch()
    A = R.laplace2d(50)
    B = np.stack([R.uniform_rhs(A.n, s) for s in (1, 2, 3)])
    h = ras.setup(A, ras.partition("regular_2d", (3, 3), grid=A.grid), 2, ras.local(loc[0], "fp64", loc[1]))
    X, infos = h.solve(_cuda(B), tol=1e-8, mode="sync", max_sweeps=100000)
    for j in range(3):
        x1, i1 = h.solve(_cuda(B[j]), tol=1e-8, mode="sync", max_sweeps=100000)
        assert torch.equal(X[j], x1)
        assert infos[j]["sweeps"] == i1[0]["sweeps"]


@pytest.mark.parametrize("kind", ["chol", "chol_sparse", "cg"])
def test_batch_equals_alone(kind):
    """Systems batched into one launch give the same iterates as alone: bit for bit
    for the direct solvers; for CG (fixed team of 2) the rows-per-thread split follows
    the largest subdomain of the launch, so sums are taken in another order and the
    iterates agree to rounding, with the same sweep counts."""
    ras = _ras()
    _say(f"case: batch {kind}")
    torch = _torch()
    A1, A2 = R.laplace2d(40), R.laplace3d(12)
    b1, b2 = R.uniform_rhs(A1.n, 3), R.uniform_rhs(A2.n, 4)
    k = 6 if kind == "cg" else 0
    team = 2 if kind == "cg" else 0
    h1 = ras.setup(A1, ras.partition("regular_2d", (2, 2), grid=A1.grid), 2, ras.local(kind, "fp64", k))
    h2 = ras.setup(A2, ras.partition("regular_3d", (2, 2, 2), grid=A2.grid), 1, ras.local(kind, "fp64", k))
    xs, infos = ras.batch_solve([h1, h2], [_cuda(b1), _cuda(b2)], tol=1e-9, mode="sync", max_sweeps=100000,
                                team=team)
    a1, i1 = h1.solve(_cuda(b1), tol=1e-9, mode="sync", max_sweeps=100000, team=team)
    a2, i2 = h2.solve(_cuda(b2), tol=1e-9, mode="sync", max_sweeps=100000, team=team)
    assert infos[0][0]["sweeps"] == i1[0]["sweeps"] and infos[1][0]["sweeps"] == i2[0]["sweeps"]
    if kind == "cg":
        _agree(xs[0].cpu().numpy(), a1.cpu().numpy(), 1e-12)
        _agree(xs[1].cpu().numpy(), a2.cpu().numpy(), 1e-12)
        # and both equal the oracle's iteration
        orc = _oracle(A1, "regular_2d", (2, 2), 2, "cg", "fp64", k)
        xo, _, ko = orc.sync(b1, 1e-9, 100000)
        assert ko == i1[0]["sweeps"]
        _agree(a1.cpu().numpy(), xo, 1e-9)
    else:
        assert torch.equal(xs[0], a1) and torch.equal(xs[1], a2)
    ys, infos = ras.batch_solve([h1, h2], [_cuda(b1), _cuda(b2)], tol=1e-9, mode="async", max_sweeps=100000,
                                team=team)
    for y, A, b in ((ys[0], A1, b1), (ys[1], A2, b2)):
        yy = y.cpu().numpy()
        assert schwarz.relative_residual(A, yy, b) < 1e-9
        assert _rel(yy, schwarz.direct_solve(A, b)) <= 1e-6


def test_batch_of_different_local_solvers_is_refused():
    """One launch runs one kernel: systems whose local solver, storage or CG
    iteration count differ cannot share a batch (RAS_E_ARG); each still solves alone."""
    ras = _ras()
    _say("case: batch mixing refused")
    A = R.laplace2d(24)
    b = _cuda(R.uniform_rhs(A.n, 36))
    part = ras.partition("regular_2d", (2, 2), grid=A.grid)
    hs = [ras.setup(A, part, 1, ras.local(*loc)) for loc in
          (("chol", "fp64"), ("cg", "fp64", 4), ("chol", "fp32"), ("cg", "fp64", 6))]
    for other in hs[1:]:
        with pytest.raises(ras.RasError) as e:
            ras.batch_solve([hs[0] if other is not hs[3] else hs[1], other], [b, b], tol=1e-8, mode="sync")
        assert e.value.status == -1
    for h in hs:
        _, info = h.solve(b, tol=1e-8, mode="sync", max_sweeps=100000)
        assert info[0]["converged"]
        h.close()


# ----------------------------------------------------------------------------- optimized Schwarz
@pytest.mark.parametrize("kind,storage,tol", [("chol", "fp64", 1e-9), ("chol_sparse", "fp64", 1e-9),
                                              ("chol", "fp32", 2e-5)])
def test_oras_matches_oracle(kind, storage, tol):
    """Robin transmission (optimized RAS): the same kernels on the modified local
    matrices reproduce the oracle's ORAS iterates, and converge in fewer sweeps than RAS."""
    ras = _ras()
    _say(f"case: oras {kind} {storage}")
    A = R.laplace2d(64)
    b = R.uniform_rhs(A.n, 1)
    part = ("regular_1d", 4)
    orc = schwarz.RAS(A, _owner(A, *part), 2, "chol", storage, robin_q=0.3)
    h = ras.setup(A, _spec(ras, A, *part), 2, ras.local(kind, storage, robin_q=0.3))
    for sweeps in (1, 3):
        xo, ho, _ = orc.sync(b, 0.0, sweeps)
        x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, tol)
    _, _, ko = orc.sync(b, 1e-8, 5000)
    x, info = h.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=5000)
    assert info[0]["converged"] and abs(info[0]["sweeps"] - ko) <= (0 if storage == "fp64" else 1)
    hr = ras.setup(A, _spec(ras, A, *part), 2, ras.local(kind, storage))
    _, ir = hr.solve(_cuda(b), tol=1e-8, mode="sync", max_sweeps=5000)
    assert info[0]["sweeps"] < ir[0]["sweeps"]
    xa, ia = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=100000, max_seconds=30)
    assert ia[0]["converged"] and schwarz.relative_residual(A, xa.cpu().numpy(), b) < 1e-8


# ----------------------------------------------------------------------------- warnings and errors
@pytest.mark.parametrize("loc,k", [("chol", 0), ("cg", 6)])
def test_not_converged_returns_valid_iterate(loc, k):
    """A limit reached before the tolerance: RAS_NOT_CONVERGED (a warning), a valid
    iterate and info; with allow_unconverged=False the binding raises it."""
    ras = _ras()
    _say(f"case: not converged {loc}")
    A = R.laplace2d(40)
    b = R.uniform_rhs(A.n, 31)
    part = ("regular_2d", (2, 2))
    orc = _oracle(A, *part, 2, loc, "fp64", k)
    h = ras.setup(A, _spec(ras, A, *part), 2, ras.local(loc, "fp64", k))
    xo, ho, _ = orc.sync(b, 1e-12, 3)
    x, info = h.solve(_cuda(b), tol=1e-12, mode="sync", max_sweeps=3)
    assert not info[0]["converged"] and info[0]["sweeps"] == 3
    _agree(x.cpu().numpy(), xo, 1e-9)
    assert abs(info[0]["rel_residual"] - schwarz.relative_residual(A, x.cpu().numpy(), b)) <= 1e-9 * ho[-1]
    with pytest.raises(ras.RasError) as e:
        h.solve(_cuda(b), tol=1e-12, mode="sync", max_sweeps=3, allow_unconverged=False)
    assert e.value.status == 1
    # asynchronous: 5 local solves per subdomain, then the exact check fails -> limit
    x, info = h.solve(_cuda(b), tol=1e-12, mode="async", max_sweeps=5, max_seconds=30)
    xx = x.cpu().numpy()
    assert not info[0]["converged"] and info[0]["max_local_solves"] == 5 and info[0]["min_local_solves"] == 5
    assert np.all(np.isfinite(xx))
    assert abs(info[0]["rel_residual"] - schwarz.relative_residual(A, xx, b)) <= 1e-9 * info[0]["rel_residual"]
    # and the residual history ends with that exact value
    _, hh = h.residual_history()
    assert hh[-1] == info[0]["rel_residual"]


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_non_finite_initial_guess_is_diverged(mode):
    """A NaN in x0 makes every residual non-finite: RAS_E_DIVERGED, in both modes."""
    ras = _ras()
    _say(f"case: diverged {mode}")
    A = R.laplace2d(40)
    b = R.uniform_rhs(A.n, 32)
    h = ras.setup(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 2, ras.local("chol", "fp64"))
    x0 = np.zeros(A.n)
    x0[A.n // 2 + 7] = np.nan
    with pytest.raises(ras.RasError) as e:
        h.solve(_cuda(b), x0=_cuda(x0), tol=1e-8, mode=mode, max_sweeps=1000, max_seconds=30)
    assert e.value.status == -7
    # the handle stays usable
    x, info = h.solve(_cuda(b), tol=1e-8, mode=mode, max_sweeps=100000, max_seconds=30)
    assert info[0]["converged"] and schwarz.relative_residual(A, x.cpu().numpy(), b) < 1e-8


def test_solve_under_a_side_stream():
    """b written on a torch side stream, solve called under that stream: the library's
    stream is ordered after it, and the result equals the default-stream solve."""
    ras = _ras()
    torch = _torch()
    _say("case: side stream")
    A = R.laplace2d(48)
    b = R.uniform_rhs(A.n, 33)
    h = ras.setup(A, ras.partition("regular_2d", (3, 3), grid=A.grid), 2, ras.local("cg", "fp64", 6))
    x_ref, _ = h.solve(_cuda(b), tol=1e-9, mode="sync", max_sweeps=100000)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        bt = torch.empty(A.n, dtype=torch.float64, device="cuda")
        bt.copy_(torch.from_numpy(b).pin_memory(), non_blocking=True)
        bt.mul_(2.0).mul_(0.5)  # more (exact) work queued on the side stream before the solve
        x, info = h.solve(bt, tol=1e-9, mode="sync", max_sweeps=100000)
    torch.cuda.synchronize()
    assert info[0]["converged"]
    assert torch.equal(x, x_ref)


def test_binding_refuses_wrong_shapes_before_any_launch():
    """The C ABI reads nrhs * n values from the addresses it is given, so the
    binding checks shapes first: a right-hand side of the wrong length or rank,
    an initial guess of another shape, a batch with a missing vector and a
    serving request of the wrong width are refused with ValueError; an initial
    guess in host memory is copied to the device."""
    ras = _ras()
    torch = _torch()
    _say("case: binding shape checks")
    A = R.laplace2d(24)
    b = R.uniform_rhs(A.n, 35)
    h = ras.setup(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol", "fp64"))
    bt = _cuda(b)
    for bad in (bt[:-1], bt.reshape(1, 1, -1), bt[:0], torch.zeros(0, A.n, dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            h.solve(bad, tol=1e-9, mode="sync")
    with pytest.raises(TypeError):
        h.solve(bt.float(), tol=1e-9, mode="sync")
    with pytest.raises(ValueError):
        h.solve(bt, x0=torch.zeros(A.n + 1, dtype=torch.float64), tol=1e-9, mode="sync")
    with pytest.raises(ValueError):
        h.relative_residual(bt, bt[:-1])
    with pytest.raises(ValueError):
        ras.batch_solve([h, h], [bt], mode="sync")
    x_ref, _ = h.solve(bt, tol=0.0, mode="sync", max_sweeps=5)
    x_host0, _ = h.solve(bt, x0=torch.zeros(A.n, dtype=torch.float64), tol=0.0, mode="sync", max_sweeps=5)
    assert x_host0.device.type == "cuda" and torch.equal(x_host0, x_ref)
    h.close()
    srv = ras.Server(1 << 30, slice_seconds=0.01)
    part = ras.partition("regular_2d", (2, 2), grid=A.grid)
    with pytest.raises(ValueError):
        srv.submit(A, part, 1, ras.local("chol", "fp64"), np.ones(A.n + 3), 1e-8)
    t = srv.submit(A, part, 1, ras.local("chol", "fp64"), np.stack([b, b]), 1e-8)
    assert srv.wait(t, 60.0)
    with pytest.raises(ValueError):
        srv.poll(t, A.n, 1)
    done, x, infos, _ = srv.poll(t, A.n, 2)
    assert done and x.shape == (2, A.n) and all(i["converged"] for i in infos)
    srv.close()


def test_autotune_picks_a_feasible_team_and_keeps_parity():
    ras = _ras()
    _say("case: autotune")
    A = R.laplace2d(90)
    b = R.uniform_rhs(A.n, 23)
    h = ras.setup(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 3, ras.local("cg", "fp64", 6))
    team, ms = h.autotune(_cuda(b), 5)
    assert team in (1, 2, 4, 8, 16) and ms > 0
    orc = _oracle(A, "regular_2d", (2, 2), 3, "cg", "fp64", 6)
    xo, _, _ = orc.sync(b, 0.0, 3)
    x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=3)  # team 0 -> the tuned one
    _agree(x.cpu().numpy(), xo, 1e-9)


# ----------------------------------------------------------------------------- full-size sampled checks
def test_config2_full_size_two_sweeps():
    """1024^2, 8x8 boxes, overlap 4, CG-10 FP64 -- the bench's launch shape."""
    ras = _ras()
    _say("case: poisson2d_1024_8x8 two sync sweeps vs oracle")
    A, b, cfg = R.config_problem("poisson2d_1024_8x8")
    orc = _oracle(A, "regular_2d", (8, 8), 4, "cg", "fp64", 10)
    xo, ho, _ = orc.sync(b, 0.0, 2)
    h = ras.setup(A, ras.partition("regular_2d", (8, 8), grid=A.grid), 4, ras.local("cg", "fp64", 10))
    x, info = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=2)
    _agree(x.cpu().numpy(), xo, 1e-9)
    _, hg = h.residual_history()
    assert np.all(np.abs(hg - ho) <= 1e-9 * ho + 1e-13)


# ----------------------------------------------------------------------------- full sizes, sampled
def _oracle_subdomain_update(A, owner, p, gamma, r, local):
    """The oracle's correction of subdomain p for the global residual r, on its
    owned points (Eq. 3, one subdomain): (owned ids, delta)."""
    from oracle import local as olocal
    from oracle import overlap as oover

    own = np.flatnonzero(owner == p)
    lay = oover.bfs_layers(A, own, gamma)
    om = np.sort(np.concatenate(lay))
    solver = olocal.LocalSolver(olocal.local_matrix(A, om), *local)
    d = solver(r[om])
    pos = np.searchsorted(om, own)
    return own, d[pos]


@pytest.mark.parametrize("kind,storage,tol", [("chol", "fp64", 1e-9), ("chol", "fp32", 2e-5), ("chol", "fp16", 2e-5),
                                              ("chol_sparse", "fp64", 1e-9)])
def test_config4_full_size_first_sweep_sampled(kind, storage, tol):
    """2048^2 diffusion, 16x16 subdomains, overlap 4, banded Cholesky (slab layout)
    or sparse Cholesky (lane streams) in the bench's launch shape (256
    workgroups): one synchronous sweep from x = 0 against the oracle's update of
    sampled subdomains (corners, edge, interior); the sparse factor solves the
    same local systems exactly (another elimination order, the same solution up to
    rounding), so the oracle's exact solve is its reference."""
    ras = _ras()
    _say(f"case: diffusion2d_2048_16x16 first sweep sampled {kind} {storage}")
    A, b, cfg = R.config_problem("diffusion2d_2048_16x16")
    h = ras.setup(A, ras.partition("regular_2d", (16, 16), grid=A.grid), 4, ras.local(kind, storage))
    x, _ = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=1)
    x = x.cpu().numpy()
    owner = opart.regular_grid(A.grid, (16, 16))
    for p in (0, 7, 136, 255):
        own, d = _oracle_subdomain_update(A, owner, p, 4, b, ("chol", storage))
        _agree(x[own], d, tol, (p, _rel(x[own], d)))


def test_config3_full_size_first_sweep_sampled():
    """128^3 Laplacian, 256 RCB subdomains (jitter 0.4), overlap 1, CG-8 FP32 with
    the autotuned team, as the bench launches it: one synchronous sweep from x = 0
    against the oracle's float32 CG-8 update of sampled subdomains."""
    ras = _ras()
    _say("case: laplace3d_128_rcb256 first sweep sampled")
    A, b, cfg = R.config_problem("laplace3d_128_rcb256")
    h = ras.setup(A, ras.partition("rcb", 256, grid=A.grid, seed=3, jitter=0.4), 1, ras.local("cg", "fp32", 8))
    bt = _cuda(b)
    team, _ = h.autotune(bt, 20)
    x, _ = h.solve(bt, tol=0.0, mode="sync", max_sweeps=1, team=team)
    x = x.cpu().numpy()
    owner = opart.rcb(A.coords(), 256, 3, 0.4)
    for p in (0, 77, 160, 255):
        own, d = _oracle_subdomain_update(A, owner, p, 1, b, ("cg", "fp32", 8))
        _agree(x[own], d, 2e-5, (p, team, _rel(x[own], d)))


@pytest.mark.gpu
def test_exact_local_autotune_picks_the_faster_and_it_converges():
    """The exact-local-solver tuner times both Cholesky solvers on the system,
    returns the faster one (the report holds both), caches the choice per
    shape, and the chosen solver reaches the tolerance with the same sweep
    count as the other (same iteration up to rounding, Sec. 3.3.1)."""
    ras = _ras()
    from paper_2003_05361_amd import autotune

    _say("case: exact local autotune 96^2 4x4")
    A = R.laplace2d(96)
    b = _cuda(R.uniform_rhs(A.n, 31))
    part = _spec(ras, A, "regular_2d", (4, 4))
    loc, rep = autotune.exact_local(A, part, 3, b, "fp64", sweeps=10)
    ms = rep["ms_per_sweep"]
    assert ms["chol"] > 0 and ms["chol_sparse"] > 0
    assert rep["choice"] == min(ms, key=ms.get) and loc["kind"] == rep["choice"]
    loc2, rep2 = autotune.exact_local(A, part, 3, b, "fp64")
    assert rep2["cached"] and loc2 == loc
    sweeps = {}
    for kind in ("chol", "chol_sparse"):
        h = ras.setup(A, part, 3, ras.local(kind, "fp64"))
        _, info = h.solve(b, tol=1e-9, mode="sync", max_sweeps=100000)
        assert info[0]["converged"]
        sweeps[kind] = info[0]["sweeps"]
        h.close()
    assert sweeps["chol"] == sweeps["chol_sparse"]
    # FP16 storage: the band is the only candidate
    _, rep16 = autotune.exact_local(A, part, 3, b, "fp16", sweeps=5)
    assert rep16["choice"] == "chol" and rep16["ms_per_sweep"]["chol_sparse"] is None


@pytest.mark.parametrize("p", [5, 0])
def test_paused_subdomain_stalls_async_until_resumed(p):
    """Host-forced stall (fault injection): a paused subdomain takes no updates,
    so the solve cannot end converged while it is stalled -- with a 1 s limit it
    returns not converged, the paused subdomain at zero local solves and every
    other one updating; resumed from another thread during the next solve, the
    iteration converges (verified).  p = 0 is the subdomain whose workgroup runs
    the detector and the time limit."""
    import threading
    import time

    ras = _ras()
    _say(f"case: paused subdomain {p}")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 41)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local("chol", "fp64"))
    h.pause(p)
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=10**9, max_seconds=1.0)
    counts = h.local_solve_counts()
    assert not info[0]["converged"] and counts[p] == 0 and np.delete(counts, p).min() > 0
    assert np.all(np.isfinite(x.cpu().numpy()))
    t = threading.Timer(0.5, lambda: h.pause(p, False))
    t.start()
    t0 = time.perf_counter()
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=10**9, max_seconds=60)
    t.join()
    assert info[0]["converged"] and time.perf_counter() - t0 >= 0.5
    assert h.local_solve_counts()[p] > 0
    assert schwarz.relative_residual(A, x.cpu().numpy(), b) < 1e-8
    h.close()


def test_cancel_stops_a_running_async_solve():
    """A cancel from another thread ends a running asynchronous solve that would
    otherwise run to its limit (tol 0): it returns not converged with a finite
    iterate well before the limit, and the next solve is not affected."""
    import threading
    import time

    ras = _ras()
    _say("case: cancel")
    A = R.laplace2d(96)
    b = R.uniform_rhs(A.n, 42)
    h = ras.setup(A, ras.partition("regular_2d", (4, 4), grid=A.grid), 3, ras.local("cg", "fp64", 6))
    t = threading.Timer(0.5, h.cancel)
    t.start()
    t0 = time.perf_counter()
    x, info = h.solve(_cuda(b), tol=0.0, mode="async", max_sweeps=10**12, max_seconds=60)
    dt = time.perf_counter() - t0
    t.join()
    assert not info[0]["converged"] and 0.4 <= dt < 20
    assert np.all(np.isfinite(x.cpu().numpy()))
    x, info = h.solve(_cuda(b), tol=1e-8, mode="async", max_sweeps=10**9, max_seconds=60)
    assert info[0]["converged"] and schwarz.relative_residual(A, x.cpu().numpy(), b) < 1e-8
    with pytest.raises(ras.RasError):
        h.pause(16)
    h.close()
