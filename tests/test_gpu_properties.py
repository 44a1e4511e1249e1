"""GPU parity on random cases (needs an MI355X): random SPD systems with a grid
pattern (graph Laplacians with edge weights over two decades plus a positive
diagonal shift), random 2-D and 3-D boxes with sides from 1, regular strips and
boxes or seeded RCB partitions, overlaps 0-3, and the float64 local solvers
(banded Cholesky, sparse Cholesky, CG-k).  The device's synchronous sweeps and
ordered (multiplicative) passes from zero equal the oracle's element by element
to 1e-9 relative (the same iteration up to rounding order; the exact solvers are
compared with the oracle's exact solve).  Derandomized: the same cases each run."""
import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import ras_inputs as R
from test_gpu_parity import _agree, _cuda, _oracle, _ras, _say, _spec

pytestmark = pytest.mark.gpu

LOCALS = [("chol", 0), ("chol_sparse", 0), ("cg", 3), ("cg", 8)]


@st.composite
def cases(draw):
    if draw(st.booleans()):
        sides = (draw(st.integers(1, 16)), draw(st.integers(1, 16)), 1)
        A = R.laplace2d(sides[0], sides[1])
    else:
        sides = (draw(st.integers(1, 6)), draw(st.integers(1, 6)), draw(st.integers(1, 6)))
        A = R.laplace3d(*sides)
    seed = draw(st.integers(0, 2**32 - 1))
    rng = np.random.default_rng(seed)
    M = sp.csr_matrix((A.data, A.indices, A.indptr), shape=(A.n, A.n))
    U = sp.triu(M, k=1).tocoo()
    W = sp.coo_matrix((-(10.0 ** rng.uniform(-1, 1, U.nnz)), (U.row, U.col)), shape=M.shape)
    W = (W + W.T).tocsr()
    S = (W + sp.diags(-np.asarray(W.sum(axis=1)).ravel() + 10.0 ** rng.uniform(-1, 0, A.n))).tocsr()
    S.sort_indices()
    A = R.CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data, A.grid)
    kind = draw(st.sampled_from(["regular_1d", "regular_grid", "rcb"]))
    if kind == "regular_1d":
        part = ("regular_1d", draw(st.integers(1, min(A.n, 8))))
    elif kind == "regular_grid":
        parts = tuple(draw(st.integers(1, min(s, 3))) for s in sides)
        part = ("regular_2d", parts[:2]) if sides[2] == 1 else ("regular_3d", parts)
    else:
        part = ("rcb", (draw(st.integers(1, min(A.n, 8))), draw(st.integers(0, 2**63 - 1)), draw(st.floats(0.0, 0.9))))
    b = rng.standard_normal(A.n)
    return A, part, draw(st.integers(0, 3)), draw(st.sampled_from(LOCALS)), draw(st.integers(1, 3)), b


@settings(max_examples=150, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(cases())
def test_random_systems_sync_and_ordered_match_the_oracle(case):
    ras = _ras()
    A, (kind, arg), gamma, (loc, k), sweeps, b = case
    _say(f"case: random n={A.n} grid={A.grid} {kind} {arg} gamma={gamma} {loc} k={k} sweeps={sweeps}")
    orc = _oracle(A, kind, arg, gamma, "chol" if loc == "chol_sparse" else loc, "fp64", k)
    xs, _, _ = orc.sync(b, 0.0, sweeps)
    xo, _ = orc.ordered(b, sweeps)
    h = ras.setup(A, _spec(ras, A, kind, arg), gamma, ras.local(loc, "fp64", k))
    try:
        x, info = h.solve(_cuda(b), tol=0.0, mode="sync", max_sweeps=sweeps)
        assert info[0]["sweeps"] == sweeps, info
        _agree(x.cpu().numpy(), xs, 1e-9, ("sync", loc, sweeps))
        x, info = h.solve(_cuda(b), tol=0.0, mode="ordered", max_sweeps=sweeps)
        _agree(x.cpu().numpy(), xo, 1e-9, ("ordered", loc, sweeps))
    finally:
        h.close()


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(cases(), st.sampled_from(["chol", "chol_sparse"]), st.sampled_from(["central", "decentral", "estimate"]))
def test_random_systems_async_converge_and_verify(case, loc, detect):
    """Asynchronous solves of the same random systems with exact local solves
    (the matrices are M-matrices: graph Laplacians plus a positive shift, for
    which asynchronous RAS converges, Sec. 2.1) reach tol 1e-8 under every
    detector, and the returned iterate's relative residual, recomputed by the
    oracle, is below tol."""
    from oracle import schwarz

    ras = _ras()
    A, (kind, arg), gamma, _, _, b = case
    _say(f"case: random async n={A.n} grid={A.grid} {kind} {arg} gamma={gamma} {loc} {detect}")
    h = ras.setup(A, _spec(ras, A, kind, arg), gamma, ras.local(loc, "fp64", 0))
    try:
        x, info = h.solve(_cuda(b), tol=1e-8, mode="async", detect=detect, max_sweeps=10**7, max_seconds=5)
        assert info[0]["converged"], info
        assert schwarz.relative_residual(A, x.cpu().numpy(), b) < 1e-8
    finally:
        h.close()
