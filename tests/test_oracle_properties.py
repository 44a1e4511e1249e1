"""Property-based pins of the oracle (CPU only): on random SPD systems with a
grid pattern (graph Laplacians with edge weights over four decades plus a
positive diagonal shift), random boxes and partitions, the oracle's RAS sweeps
are checked against the mathematics, built here densely and independently of
the oracle's own overlap and local-matrix code:
  - one sweep of restricted additive Schwarz (Sec. 2.1) from x is
    x + sum_p Rt_p^T A_p^{-1} R_p (b - A x), with Omega_p grown by gamma
    applications of the pattern of A (matrix powers) and Rt_p the restriction
    to the owned points;
  - without overlap a sweep is block Jacobi and an ordered pass block
    Gauss-Seidel over the owned blocks;
  - one subdomain gives the direct solve in one sweep."""
import numpy as np
import scipy.sparse as sp
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import ras_inputs as R
from oracle import partition as opart
from oracle import schwarz


@st.composite
def systems(draw):
    if draw(st.booleans()):
        grid = (draw(st.integers(1, 14)), draw(st.integers(1, 14)), 1)
        A = R.laplace2d(grid[0], grid[1])
    else:
        grid = (draw(st.integers(1, 6)), draw(st.integers(1, 6)), draw(st.integers(1, 6)))
        A = R.laplace3d(*grid)
    rng = np.random.default_rng(draw(st.integers(0, 2**32 - 1)))
    M = sp.csr_matrix((A.data, A.indices, A.indptr), shape=(A.n, A.n))
    U = sp.triu(M, k=1).tocoo()
    W = sp.coo_matrix((-(10.0 ** rng.uniform(-2, 2, U.nnz)), (U.row, U.col)), shape=M.shape)
    W = (W + W.T).tocsr()
    S = (W + sp.diags(-np.asarray(W.sum(axis=1)).ravel() + 10.0 ** rng.uniform(-2, 0, A.n))).tocsr()
    S.sort_indices()
    A = R.CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data, A.grid)
    if draw(st.booleans()):
        owner = opart.regular_1d(A.n, draw(st.integers(1, min(A.n, 8))))
    else:
        owner = opart.rcb(A.coords(), draw(st.integers(1, min(A.n, 8))), draw(st.integers(0, 2**63 - 1)),
                          draw(st.floats(0.0, 0.9)))
    b = rng.standard_normal(A.n)
    x0 = rng.standard_normal(A.n)
    return A, S.toarray(), owner, b, x0


def _omega(D, owned, gamma):
    """Omega_p: the owned points grown by gamma applications of A's pattern."""
    reach = np.zeros(D.shape[0], dtype=bool)
    reach[owned] = True
    pattern = D != 0
    for _ in range(gamma):
        reach = reach | pattern[reach].any(axis=0)
    return np.flatnonzero(reach)


def _ras_sweep(D, owner, gamma, b, x):
    r = b - D @ x
    x1 = x.copy()
    for p in range(int(owner.max()) + 1):
        owned = np.flatnonzero(owner == p)
        om = _omega(D, owned, gamma)
        delta = np.linalg.solve(D[np.ix_(om, om)], r[om])
        keep = np.isin(om, owned)
        x1[om[keep]] += delta[keep]
    return x1


@settings(max_examples=80, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(systems(), st.integers(0, 3))
def test_sync_sweep_is_the_ras_update(sysm, gamma):
    A, D, owner, b, x0 = sysm
    orc = schwarz.RAS(A, owner, gamma, "chol", "fp64", 0)
    x1, _, sweeps = orc.sync(b, 0.0, 1, x0=x0)
    assert sweeps == 1
    ref = _ras_sweep(D, owner, gamma, b, x0)
    assert np.max(np.abs(x1 - ref)) <= 1e-9 * max(np.max(np.abs(ref)), 1.0)


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(systems())
def test_no_overlap_is_block_jacobi_and_block_gauss_seidel(sysm):
    A, D, owner, b, x0 = sysm
    P = int(owner.max()) + 1
    blocks = [np.flatnonzero(owner == p) for p in range(P)]
    jac = x0.copy()
    for o in blocks:
        jac[o] = np.linalg.solve(D[np.ix_(o, o)], b[o] - D[o] @ x0 + D[np.ix_(o, o)] @ x0[o])
    gs = x0.copy()
    for o in blocks:
        gs[o] = np.linalg.solve(D[np.ix_(o, o)], b[o] - D[o] @ gs + D[np.ix_(o, o)] @ gs[o])
    orc = schwarz.RAS(A, owner, 0, "chol", "fp64", 0)
    xj, _, _ = orc.sync(b, 0.0, 1, x0=x0)
    xg, _ = orc.ordered(b, 1, x0=x0)
    scale = max(np.max(np.abs(jac)), np.max(np.abs(gs)), 1.0)
    assert np.max(np.abs(xj - jac)) <= 1e-9 * scale
    assert np.max(np.abs(xg - gs)) <= 1e-9 * scale


@settings(max_examples=40, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(systems(), st.integers(0, 3))
def test_one_subdomain_is_the_direct_solve(sysm, gamma):
    A, D, _, b, x0 = sysm
    orc = schwarz.RAS(A, np.zeros(A.n, dtype=np.int32), gamma, "chol", "fp64", 0)
    x1, _, _ = orc.sync(b, 0.0, 1, x0=x0)
    xd = np.linalg.solve(D, b)
    assert np.max(np.abs(x1 - xd)) <= 1e-9 * max(np.max(np.abs(xd)), 1.0)


def _krylov_basis(D, r, k):
    """Orthonormal basis of K_k(D, r) by Arnoldi with one reorthogonalisation;
    stops early where the space becomes invariant."""
    V = [r / np.linalg.norm(r)]
    for _ in range(k - 1):
        w = D @ V[-1]
        for _ in range(2):
            for v in V:
                w = w - (v @ w) * v
        nw = np.linalg.norm(w)
        if nw <= 1e-10 * np.linalg.norm(D @ V[-1]):
            break
        V.append(w / nw)
    return np.stack(V, axis=1)


@settings(max_examples=80, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(systems(), st.integers(1, 5), st.integers(0, 3))
def test_cg_steps_are_the_krylov_galerkin_projection(sysm, k, gamma):
    """The oracle's CG-k local solve from zero (Sec. 3.3.1, inexact local solves)
    is the A_p-orthogonal projection of A_p^{-1} r onto K_k(A_p, r):
    V (V^T A_p V)^{-1} V^T r, for the local matrix of a random subdomain."""
    from oracle import local as olocal

    A, D, owner, b, x0 = sysm
    om = _omega(D, np.flatnonzero(owner == 0), gamma)
    Dp = D[np.ix_(om, om)]
    r = (b - D @ x0)[om]
    V = _krylov_basis(Dp, r, k)
    ref = V @ np.linalg.solve(V.T @ Dp @ V, V.T @ r)
    d = olocal.cg_fixed(sp.csr_matrix(Dp), r, k)
    assert np.linalg.norm(d - ref) <= 1e-8 * np.linalg.norm(ref)


@settings(max_examples=150, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(1, 12), st.integers(1, 9), st.integers(0, 2**32 - 1), st.booleans())
def test_compensated_residual_within_the_dot2_bound(rows, per_row, seed, cancel):
    """The oracle's outer residual b - A x is Dot2 (Ogita, Rump, Oishi 2005): for
    each row of m = per_row + 1 terms, |res - exact| <= eps |exact| +
    gamma_m^2 (|b_i| + sum_j |a_ij x_j|) with eps = 2^-53 and gamma_m = m eps /
    (1 - m eps); the exact value in rational arithmetic.  With `cancel`, b is
    the float64 product A x plus a few ulps, so the residual cancels almost
    completely (where plain float64 is off by about the size of r itself)."""
    from fractions import Fraction

    from oracle import residual as oresidual

    rng = np.random.default_rng(seed)
    n = 40
    indptr = [0]
    cols, vals = [], []
    for _ in range(rows):
        c = np.sort(rng.choice(n, size=per_row, replace=False))
        cols.extend(c.tolist())
        vals.extend((rng.standard_normal(per_row) * 2.0 ** rng.integers(-30, 30, per_row)).tolist())
        indptr.append(len(cols))
    M = sp.csr_matrix((np.array(vals), np.array(cols, dtype=np.int32), np.array(indptr, dtype=np.int64)),
                      shape=(rows, n))
    x = rng.standard_normal(n) * 2.0 ** rng.integers(-20, 20, n)
    b = np.zeros(n)
    b[:rows] = (M @ x) * (1.0 + rng.integers(-3, 4, rows) * 2.0 ** -52) if cancel else rng.standard_normal(rows)
    r = oresidual.residual(M, x, b)
    eps = 2.0 ** -53
    gamma = (per_row + 1) * eps / (1 - (per_row + 1) * eps)
    for i in range(rows):
        lo_, hi_ = indptr[i], indptr[i + 1]
        exact = Fraction(b[i]) - sum(Fraction(vals[k]) * Fraction(x[cols[k]]) for k in range(lo_, hi_))
        size = abs(b[i]) + sum(abs(vals[k] * x[cols[k]]) for k in range(lo_, hi_))
        err = abs(Fraction(r[i]) - exact)
        assert err <= Fraction(eps) * abs(exact) + Fraction(gamma * gamma * size * 1.01), (i, float(err), float(exact))
