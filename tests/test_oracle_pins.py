"""Pins of the oracle against the mathematics and the paper (CPU only).

Each test checks the oracle against something other than itself: a direct
solve, an independently built operator, a closed form, a brute-force index
set, or a value written out from the paper.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import ras_inputs as R
from oracle import local, overlap, partition, schwarz

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- problems (Sec. 4.1)
def test_generator_matches_paper_stencil():
    """The 2-D generator reproduces the hand-written 3x3 operator of the paper's stencil."""
    ref = np.loadtxt(os.path.join(GOLDEN, "laplace2d_3x3.txt"))
    assert np.array_equal(R.laplace2d(3).scipy().toarray(), ref)


def test_sine_modes_are_eigenpairs():
    A = R.laplace2d(9, 9)
    v, lam = R.sine_mode_2d(9, 2, 5)
    assert np.linalg.norm(A.matvec(v) - lam * v) <= 1e-13 * np.linalg.norm(v)
    A3 = R.laplace3d(6)
    v3, lam3 = R.sine_mode_3d(6, 1, 2, 4)
    assert np.linalg.norm(A3.matvec(v3) - lam3 * v3) <= 1e-13 * np.linalg.norm(v3)


def test_tpfa_is_symmetric_m_matrix():
    g = R.gaussian_random_field_2d(32, 4.0, 11)
    A = R.tpfa2d(np.exp(2 * g), 10.0).scipy()
    assert abs(A - A.T).max() == 0
    off = A - sp.diags(A.diagonal())
    assert off.max() <= 0
    # strictly diagonally dominant on wall cells, weakly inside -> SPD
    assert np.all(A.diagonal() + np.asarray(off.sum(axis=1)).ravel() >= -1e-12)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


# ----------------------------------------------------------------- P1: one subdomain
@pytest.mark.parametrize("local_kind", ["chol", "cg"])
def test_single_subdomain_is_direct_solve(local_kind):
    A = R.laplace2d(12, 10)
    b = R.uniform_rhs(A.n, 3)
    owner = np.zeros(A.n, dtype=np.int32)
    ras = schwarz.RAS(A, owner, 0, local_kind, "fp64", cg_iters=A.n)
    x, hist, k = ras.sync(b, 1e-12, 1)
    xd = np.linalg.solve(A.scipy().toarray(), b)
    assert k == 1
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd) * (1e2 if local_kind == "cg" else 1)
    assert hist[1] <= 1e-11


# ----------------------------------------------------------------- P2: zero overlap = block Jacobi
def test_zero_overlap_is_block_jacobi():
    A = R.laplace2d(12)
    b = R.uniform_rhs(A.n, 4)
    owner = partition.regular_grid(A.grid, (3, 2))
    ras = schwarz.RAS(A, owner, 0, "chol")
    M = A.scipy().tocoo()
    same = owner[M.row] == owner[M.col]
    D = sp.csc_matrix((M.data[same], (M.row[same], M.col[same])), shape=M.shape)
    lu = spla.splu(D)
    x = np.zeros(A.n)
    for k in range(1, 6):
        x = x + lu.solve(b - A.matvec(x))
        xo, _, kk = ras.sync(b, 0.0, k)
        assert kk == k
        assert np.linalg.norm(xo - x) <= 1e-13 * np.linalg.norm(x)


# ----------------------------------------------------------------- P3: manufactured sine modes
def test_sine_mode_solution_and_strip_invariant():
    N = 24
    A = R.laplace2d(N)
    v, lam = R.sine_mode_2d(N, 1, 1)
    b = lam * v
    owner = partition.regular_1d(A.n, 4)
    ras = schwarz.RAS(A, owner, 2, "chol")
    # invariant: with row strips the x-profile of every iterate is the sine mode
    for k in (1, 2, 5):
        xk, _, _ = ras.sync(b, 0.0, k)
        X = xk.reshape(N, N)  # [j, i]
        sx = np.sin(np.pi * np.arange(1, N + 1) / (N + 1))
        proj = np.outer(X @ sx / (sx @ sx), sx)
        assert np.linalg.norm(X - proj) <= 1e-12 * np.linalg.norm(X)
    x, hist, _ = ras.sync(b, 1e-10, 5000)
    assert hist[-1] < 1e-10
    assert np.linalg.norm(x - v) <= 1e-6 * np.linalg.norm(v)


def test_sine_mode_3d():
    N = 10
    A = R.laplace3d(N)
    v, lam = R.sine_mode_3d(N, 1, 1, 1)
    owner = partition.regular_grid(A.grid, (2, 2, 2))
    ras = schwarz.RAS(A, owner, 1, "chol")
    x, hist, _ = ras.sync(lam * v, 1e-10, 5000)
    assert np.linalg.norm(x - v) <= 1e-6 * np.linalg.norm(v)


# ----------------------------------------------------------------- P4: iteration operator
def _dense_operator(A, owner, gamma):
    """T = I - sum_p Rt_p^T A_p^{-1} R_p A, built from dense selection matrices."""
    n = A.n
    Ad = A.scipy().toarray()
    Ms = np.zeros((n, n))
    reach = np.eye(n) + (np.abs(Ad) > 0)
    for p in range(owner.max() + 1):
        ind = (owner == p).astype(float)
        for _ in range(gamma):
            ind = (reach @ ind > 0).astype(float)
        om = np.flatnonzero(ind)
        Rp = np.zeros((om.size, n))
        Rp[np.arange(om.size), om] = 1.0
        Rt = Rp.copy()
        Rt[owner[om] != p, :] = 0.0
        Ms += Rt.T @ np.linalg.inv(Rp @ Ad @ Rp.T) @ Rp
    return np.eye(n) - Ms @ Ad


def test_iteration_operator():
    A = R.laplace2d(14, 12)
    owner = partition.regular_grid(A.grid, (2, 2))
    gamma = 2
    T = _dense_operator(A, owner, gamma)
    ras = schwarz.RAS(A, owner, gamma, "chol")
    b = R.uniform_rhs(A.n, 5)
    xs = np.linalg.solve(A.scipy().toarray(), b)
    e_prev = -xs
    for k in range(1, 8):
        xk, _, _ = ras.sync(b, 0.0, k)
        e = xk - xs
        assert np.linalg.norm(e - T @ e_prev) <= 1e-12 * np.linalg.norm(xs)
        e_prev = e
    ev = np.linalg.eigvals(T)
    rho = np.abs(ev).max()
    assert rho < 1
    top = ev[np.argsort(-np.abs(ev))[:2]]
    if abs(top[0].imag) < 1e-12 and abs(abs(top[0]) - abs(top[1])) > 1e-3:
        _, hist, _ = ras.sync(b, 0.0, 16)
        assert abs(hist[16] / hist[15] - rho) <= 1e-6


# ----------------------------------------------------------------- P5: index sets
def test_regular_partitions_closed_form():
    o1 = partition.regular_1d(64 * 64, 4)
    assert np.array_equal(np.bincount(o1), [1024] * 4)
    assert np.all(np.diff(o1) >= 0)
    A = R.laplace2d(10, 7)
    o2 = partition.regular_grid(A.grid, (3, 2))
    X = o2.reshape(7, 10)
    # x slabs [0,3) [3,6) [6,10); y slabs [0,3) [3,7)
    expect = np.zeros((7, 10), dtype=int)
    for j in range(7):
        for i in range(10):
            expect[j, i] = (0 if i < 3 else 1 if i < 6 else 2) + 3 * (0 if j < 3 else 1)
    assert np.array_equal(X, expect)


@pytest.mark.parametrize("gamma", [0, 1, 2, 3])
def test_overlap_matches_matrix_powers(gamma):
    A = R.laplace2d(11, 9)
    owner = partition.regular_grid(A.grid, (3, 2))
    sets = overlap.subdomain_sets(A, owner, gamma)
    G = (sp.identity(A.n) + abs(A.scipy())).tocsr()
    G.data[:] = 1.0
    for p, (own, om, ext) in enumerate(sets):
        v = (owner == p).astype(float)
        for _ in range(gamma):
            v = G @ v
        ref = np.flatnonzero(v > 0)
        assert np.array_equal(om, ref)
        ref_ext = np.setdiff1d(np.flatnonzero(G @ v > 0), ref)
        assert np.array_equal(ext, ref_ext)
        assert np.array_equal(own, np.flatnonzero(owner == p))


def test_overlap_config1_sizes():
    """Strips of 16 grid rows with two rows of overlap: 18 or 20 rows of 64."""
    A = R.laplace2d(64)
    sets = overlap.subdomain_sets(A, partition.regular_1d(A.n, 4), 2)
    assert [om.size for _, om, _ in sets] == [18 * 64, 20 * 64, 20 * 64, 18 * 64]


# ----------------------------------------------------------------- communication volume (Fig. 2)
def test_comm_volume_strips_closed_form():
    """Strips of t grid lines of an N-wide grid: with gamma + 1 <= t, each strip
    reads gamma overlap lines plus one external line from each neighbour."""
    N, P = 24, 4
    A = R.laplace2d(N)
    owner = partition.regular_1d(A.n, P)
    for gamma in (0, 1, 2, 5):
        vol = overlap.comm_volume(owner, overlap.subdomain_sets(A, owner, gamma))
        expect = np.zeros((P, P), dtype=np.int64)
        for p in range(P - 1):
            expect[p, p + 1] = expect[p + 1, p] = (gamma + 1) * N
        assert np.array_equal(vol, expect), gamma


def _manhattan_volume(A, owner, gamma):
    """Brute force over a full grid with the 5/7-point stencil: graph distance from
    a point to a set is the least Manhattan distance to it, so p needs every point
    of another subdomain that lies within gamma + 1 of O_p."""
    X = A.coords()
    P = int(owner.max()) + 1
    vol = np.zeros((P, P), dtype=np.int64)
    for p in range(P):
        own = X[owner == p]
        d = np.abs(X[:, None, :] - own[None, :, :]).sum(axis=2).min(axis=1)
        for i in np.flatnonzero((d <= gamma + 1) & (owner != p)):
            vol[p, owner[i]] += 1
    return vol


@pytest.mark.parametrize("gamma", [0, 1, 2, 3])
def test_comm_volume_matches_manhattan_brute_force(gamma):
    cases = [
        (R.laplace2d(13, 11), partition.regular_grid((13, 11, 1), (3, 2))),
        (R.laplace2d(12), partition.regular_1d(144, 5)),  # strip boundaries off the grid lines
        (R.laplace2d(14, 9), partition.rcb(R.laplace2d(14, 9).coords(), 6, 4, 0.3)),
        (R.laplace3d(6), partition.regular_grid((6, 6, 6), (2, 3, 2))),
    ]
    for A, owner in cases:
        vol = overlap.comm_volume(owner, overlap.subdomain_sets(A, owner, gamma))
        assert np.array_equal(vol, _manhattan_volume(A, owner, gamma))


def test_comm_volume_blocks_closed_form():
    """Blocks of bx x by with gamma + 1 <= min(bx, by): an edge neighbour gives a
    (gamma + 1)-deep slab along the shared side, a corner neighbour the lattice
    points (dx, dy >= 1, dx + dy <= gamma + 1), gamma (gamma + 1) / 2 of them."""
    A = R.laplace2d(24, 30)  # 3 x 2 blocks of 8 x 15
    owner = partition.regular_grid(A.grid, (3, 2))
    gamma = 3
    vol = overlap.comm_volume(owner, overlap.subdomain_sets(A, owner, gamma))
    bx, by = 8, 15
    for p in range(6):
        for q in range(6):
            dxb = abs(p % 3 - q % 3)
            dyb = abs(p // 3 - q // 3)
            if p == q or dxb > 1 or dyb > 1:
                e = 0
            elif dyb == 0:
                e = (gamma + 1) * by
            elif dxb == 0:
                e = (gamma + 1) * bx
            else:
                e = gamma * (gamma + 1) // 2
            assert vol[p, q] == e, (p, q)


def _rcb_literal(coords, ids, p0, m, w, out):
    if m == 1:
        for g in ids:
            out[g] = p0
        return
    ml = m // 2
    ext = [max(coords[g][a] for g in ids) - min(coords[g][a] for g in ids) for a in range(3)]
    axis = ext.index(max(ext))
    ids = sorted(ids, key=lambda g: (coords[g][axis], g))
    Wl = sum(w[p0:p0 + ml])
    W = sum(w[p0:p0 + m])
    cut = math.floor(len(ids) * Wl / W + 0.5)
    cut = min(max(cut, ml), len(ids) - (m - ml))
    _rcb_literal(coords, ids[:cut], p0, ml, w, out)
    _rcb_literal(coords, ids[cut:], p0 + ml, m - ml, w, out)


@pytest.mark.parametrize("shape,P,seed", [((9, 7, 1), 5, 3), ((6, 5, 4), 7, 11), ((12, 12, 1), 16, 0)])
def test_rcb_matches_literal_version(shape, P, seed):
    A = R.laplace2d(shape[0], shape[1]) if shape[2] == 1 else R.laplace3d(shape[0])
    coords = A.coords()
    owner = partition.rcb(coords, P, seed, 0.4)
    ref = [-1] * A.n
    w = partition.rcb_weights(P, seed, 0.4)
    _rcb_literal([tuple(c) for c in coords], list(range(A.n)), 0, P, w, ref)
    assert np.array_equal(owner, np.array(ref))
    assert set(owner.tolist()) == set(range(P))


def test_splitmix64_published_vectors():
    rows = np.loadtxt(os.path.join(GOLDEN, "splitmix64_vectors.txt"), dtype=np.uint64)
    for seed, idx, val in rows:
        assert partition.splitmix64_outputs(int(seed), int(idx) + 1)[-1] == int(val)


def test_rcb_weights_in_range():
    w = partition.rcb_weights(256, 3, 0.4)
    assert min(w) >= 0.6 and max(w) <= 1.4 and len(set(w)) == 256


# ----------------------------------------------------------------- P6: local CG
def _spd_local(n=40, seed=0):
    A = R.tpfa2d(np.exp(R.gaussian_random_field_2d(8, 2.0, seed)[:5, :8]))
    return A.scipy()


def test_cg_full_length_is_exact():
    Ap = _spd_local()
    r = np.random.default_rng(1).standard_normal(Ap.shape[0])
    d = local.cg_fixed(Ap, r, 4 * Ap.shape[0])
    assert np.linalg.norm(d - spla.spsolve(Ap.tocsc(), r)) <= 1e-10 * np.linalg.norm(d)


def test_cg_one_step_is_steepest_descent():
    Ap = _spd_local()
    r = np.random.default_rng(2).standard_normal(Ap.shape[0])
    d = local.cg_fixed(Ap, r, 1)
    assert np.allclose(d, (r @ r) / (r @ (Ap @ r)) * r, rtol=1e-14, atol=0)


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_cg_is_krylov_galerkin_projection(k):
    """CG-k minimises the A-norm error over K_k(A, r): delta = V (V'AV)^{-1} V' r."""
    Ap = _spd_local().toarray()
    r = np.random.default_rng(3).standard_normal(Ap.shape[0])
    K = np.stack([np.linalg.matrix_power(Ap, j) @ r for j in range(k)], axis=1)
    V, _ = np.linalg.qr(K)
    ref = V @ np.linalg.solve(V.T @ Ap @ V, V.T @ r)
    d = local.cg_fixed(sp.csr_matrix(Ap), r, k)
    assert np.linalg.norm(d - ref) <= 1e-9 * np.linalg.norm(ref)


def test_cg_fp32_tracks_fp64():
    Ap = _spd_local()
    r = np.random.default_rng(4).standard_normal(Ap.shape[0])
    d64 = local.cg_fixed(Ap, r, 8)
    d32 = local.cg_fixed(Ap, r, 8, np.float32)
    assert np.linalg.norm(d32 - d64) <= 1e-4 * np.linalg.norm(d64)
    assert not np.array_equal(d32, d64)


# ----------------------------------------------------------------- P7: band Cholesky
def test_band_cholesky_factor():
    A = R.laplace2d(9, 6)
    omega = overlap.subdomain_sets(A, partition.regular_1d(A.n, 2), 1)[0][1]
    Ap = local.local_matrix(A, omega)
    cb, w = local.band_cholesky(Ap)
    assert w == 9
    L = local.band_to_dense_lower(cb)
    Ad = Ap.toarray()
    assert np.linalg.norm(L @ L.T - Ad) <= 1e-14 * np.linalg.norm(Ad)
    assert np.allclose(L, np.linalg.cholesky(Ad), rtol=0, atol=1e-14)
    r = np.random.default_rng(0).standard_normal(Ap.shape[0])
    assert np.allclose(local.chol_solve_fp64(cb, r), np.linalg.solve(Ad, r), rtol=1e-13, atol=1e-13)


def test_reduced_precision_factor():
    g = R.gaussian_random_field_2d(16, 3.0, 9)
    A = R.tpfa2d(np.exp(2 * g), 10.0)
    Ap = A.scipy()
    cb, w = local.band_cholesky(Ap)
    L = local.band_to_dense_lower(cb)
    Lhat, s = local.quantize_rows_fp16(cb)
    Lh = local.band_to_dense_lower(Lhat.astype(np.float64))
    assert np.abs(Lh).max() <= 1.0
    # every stored entry is within half an fp16 ulp of L/s, relative to the row scale
    rel = np.abs(Lh * s.astype(np.float64)[:, None] - L) / s.astype(np.float64)[:, None]
    assert rel.max() <= 2.0 ** -11 * (1 + 1e-6)
    r = np.random.default_rng(5).standard_normal(A.n)
    x64 = np.linalg.solve(Ap.toarray(), r)
    for st, bound in (("fp32", 1e-3), ("fp16", 0.5)):
        x = local.LocalSolver(Ap, "chol", st)(r)
        assert np.linalg.norm(x - x64) <= bound * np.linalg.norm(x64)
        assert not np.array_equal(x, x64)


# ----------------------------------------------------------------- P8: information propagation (Sec. 3.2.1)
def test_regular1d_information_propagation():
    N, P, gamma = 16, 4, 1  # strips of 4 rows > gamma
    A = R.laplace2d(N)
    owner = partition.regular_1d(A.n, P)
    b = np.zeros(A.n)
    b[N * 0 + 5] = 1.0  # row 0 of strip 0: farther than gamma from strip 1
    ras = schwarz.RAS(A, owner, gamma, "chol")
    for k in range(1, P + 1):
        xk, _, _ = ras.sync(b, 0.0, k)
        reached = sorted(set(owner[np.flatnonzero(xk != 0.0)].tolist()))
        assert reached == list(range(k))


# ----------------------------------------------------------------- P9: monotonicity (Sec. 4.3, Sec. 3.2.1)
def test_more_overlap_fewer_sweeps():
    A = R.laplace2d(32)
    b = R.uniform_rhs(A.n, 6)
    sweeps = []
    for gamma in (1, 2, 4):
        ras = schwarz.RAS(A, partition.regular_1d(A.n, 4), gamma, "chol")
        sweeps.append(ras.sync(b, 1e-8, 10000)[2])
    assert sweeps[0] >= sweeps[1] >= sweeps[2]
    r1 = schwarz.RAS(A, partition.regular_1d(A.n, 16), 2, "chol").sync(b, 1e-8, 10000)[2]
    r2 = schwarz.RAS(A, partition.regular_grid(A.grid, (4, 4)), 2, "chol").sync(b, 1e-8, 10000)[2]
    assert r2 < r1


def test_sync_with_thread_pool_is_the_same_iteration():
    """The local solves of one synchronous sweep all read r^k: running them on a
    thread pool (the all-cores CPU baseline) gives the same iterates bit for bit."""
    import concurrent.futures as cf

    A = R.laplace2d(40)
    b = R.uniform_rhs(A.n, 9)
    for loc, k in (("chol", 0), ("cg", 5)):
        ras = schwarz.RAS(A, partition.regular_grid(A.grid, (3, 3)), 2, loc, "fp64", k)
        x1, h1, k1 = ras.sync(b, 0.0, 6)
        with cf.ThreadPoolExecutor(4) as pool:
            x2, h2, k2 = ras.sync(b, 0.0, 6, pool=pool)
        assert k1 == k2 == 6 and np.array_equal(x1, x2) and np.array_equal(h1, h2)


# ----------------------------------------------------------------- outer residual (Sec. 3.3.2)
def _exact_residual(M, x, b):
    """b - M x in exact rational arithmetic, rounded once to float64."""
    from fractions import Fraction

    out = np.empty(M.shape[0])
    for i in range(M.shape[0]):
        acc = Fraction(float(b[i]))
        for e in range(M.indptr[i], M.indptr[i + 1]):
            acc -= Fraction(float(M.data[e])) * Fraction(float(x[M.indices[e]]))
        out[i] = float(acc)
    return out


def test_error_free_transformations_are_exact():
    from fractions import Fraction

    from oracle import residual as ores

    rng = np.random.default_rng(40)
    a = rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 9, 2000)
    c = rng.standard_normal(2000) * 10.0 ** rng.integers(-8, 9, 2000)
    p, e = ores.two_product(a, c)
    s, t = ores.two_sum(a, c)
    for i in range(2000):
        assert Fraction(p[i]) + Fraction(e[i]) == Fraction(a[i]) * Fraction(c[i])
        assert Fraction(s[i]) + Fraction(t[i]) == Fraction(a[i]) + Fraction(c[i])
        assert p[i] == a[i] * c[i] and s[i] == a[i] + c[i]


def test_compensated_residual_against_exact_arithmetic():
    """Where b - A x cancels (b = fl(A x), log-normal coefficients, |x| ~ 1e4), the
    compensated residual meets Dot2's bound |r^ - r| <= u |r| + gamma_n^2 (|b| + |A||x|)
    against the exact rational residual, while a plain float64 evaluation is off by
    about u (|A||x|), i.e. by the size of r itself."""
    from oracle import residual as ores

    g = R.gaussian_random_field_2d(24, 4.0, 41)
    A = R.tpfa2d(np.exp(2.0 * g), 10.0)
    M = A.scipy()
    rng = np.random.default_rng(42)
    x = rng.uniform(-1.0, 1.0, A.n) * 1e4
    b = M @ x  # plain float64: the exact residual is the rounding error of this product
    r_exact = _exact_residual(M, x, b)
    r_comp = ores.residual(M, x, b)
    u = 2.0 ** -53
    n = int(np.diff(M.indptr).max()) + 1
    gamma = n * u / (1 - n * u)
    mag = np.abs(b) + np.abs(M) @ np.abs(x)
    assert np.all(np.abs(r_comp - r_exact) <= u * np.abs(r_exact) + gamma ** 2 * mag)
    # the case has teeth: plain float64 misses rows by far more than the bound
    r_plain = b - M @ x
    assert np.max(np.abs(r_plain - r_exact) / mag) > 1e3 * gamma ** 2
    # a subset of rows gives the same values as the full evaluation
    rows = np.arange(3, A.n, 7)
    assert np.array_equal(ores.residual(M, x, b, rows), r_comp[rows])


def test_relative_residual_of_an_exact_solution():
    """An exactly representable solution: x integer, b = A x exactly (integer
    coefficients): the compensated residual is exactly zero."""
    A = R.laplace2d(20)
    x = np.random.default_rng(43).integers(-1000, 1000, A.n).astype(np.float64)
    b = A.scipy() @ x
    assert schwarz.relative_residual(A, x, b) == 0.0


# ----------------------------------------------------------------- optimized Schwarz (Robin transmission)
def test_robin_with_q_one_is_ras():
    A = R.laplace2d(30)
    b = R.uniform_rhs(A.n, 44)
    owner = partition.regular_grid(A.grid, (2, 3))
    x1, h1, _ = schwarz.RAS(A, owner, 2, "chol").sync(b, 0.0, 5)
    x2, h2, _ = schwarz.RAS(A, owner, 2, "chol", robin_q=1.0).sync(b, 0.0, 5)
    assert np.array_equal(x1, x2) and np.array_equal(h1, h2)


def test_robin_local_matrix_by_hand():
    """5-point 2-D Laplacian, 4 x 4 grid, two 1-D strips, no overlap: the first strip's
    rows 4..7 each couple to one point outside (|a| = 1), so their diagonal 4 becomes
    4 - (1 - q); rows 0..3 keep 4; off-diagonals are unchanged."""
    A = R.laplace2d(4)
    om = np.arange(8)
    q = 0.25
    Ap = local.robin_local_matrix(A, om, q).toarray()
    ref = A.scipy().toarray()[:8, :8].copy()
    ref[np.arange(4, 8), np.arange(4, 8)] = 4.0 - 0.75
    assert np.array_equal(Ap, ref)
    assert np.array_equal(local.outside_coupling(A, om), np.array([0, 0, 0, 0, 1, 1, 1, 1.0]))


@pytest.mark.parametrize("gamma", [1, 3])
def test_optimal_robin_two_subdomains_exact_after_two_sweeps(gamma):
    """With transparent transmission (the exact Schur complement of the outside part,
    which for a tridiagonal matrix only changes the boundary row's diagonal), two
    overlapping subdomains of a 1-D problem give the exact solution after two sweeps
    (the optimal Schwarz method, Gander 2006).  The oracle's Robin form lowers the
    diagonal by (1 - q) e_i; here q is chosen per subdomain so that the lowered
    diagonal equals the Schur complement's."""
    n = 40
    A = R.laplace2d(n, 1)  # tridiag(-1, 4, -1)
    M = A.scipy().toarray()
    owner = partition.regular_1d(n, 2)
    b = R.uniform_rhs(n, 45)
    orc = schwarz.RAS(A, owner, gamma, "chol")
    for sd in orc.subs:
        out = np.setdiff1d(np.arange(n), sd.omega)
        schur = M[np.ix_(sd.omega, out)] @ np.linalg.solve(M[np.ix_(out, out)], M[np.ix_(out, sd.omega)])
        e = local.outside_coupling(A, sd.omega)
        i = int(np.flatnonzero(e)[0])  # the one boundary row
        q = 1.0 - schur[i, i] / e[i]
        Ap = local.robin_local_matrix(A, sd.omega, q)
        assert np.allclose(Ap.toarray(), M[np.ix_(sd.omega, sd.omega)] - schur, atol=1e-15)
        sd.solver = local.LocalSolver(Ap, "chol")
    _, hist, _ = orc.sync(b, 0.0, 3)
    assert hist[1] > 1e-4 and hist[2] < 1e-14 and hist[3] < 1e-14


def test_robin_reduces_sweeps_on_strips():
    A = R.laplace2d(64)
    b = R.uniform_rhs(A.n, 1)
    owner = partition.regular_1d(A.n, 4)
    k_ras = schwarz.RAS(A, owner, 2, "chol").sync(b, 1e-8, 3000)[2]
    k_oras = schwarz.RAS(A, owner, 2, "chol", robin_q=0.1).sync(b, 1e-8, 3000)[2]
    assert k_ras == 113 and k_oras < k_ras / 3
    x = schwarz.RAS(A, owner, 2, "chol", robin_q=0.1).sync(b, 1e-10, 3000)[0]
    assert np.linalg.norm(x - schwarz.direct_solve(A, b)) <= 1e-8 * np.linalg.norm(x)


# ----------------------------------------------------------------- P10: ordered / asynchronous
def test_ordered_zero_overlap_is_block_gauss_seidel():
    A = R.laplace2d(12)
    b = R.uniform_rhs(A.n, 7)
    owner = partition.regular_grid(A.grid, (2, 3))
    M = A.scipy().tocoo()
    low = owner[M.col] <= owner[M.row]
    DL = sp.csc_matrix((M.data[low], (M.row[low], M.col[low])), shape=M.shape)
    lu = spla.splu(DL)
    ras = schwarz.RAS(A, owner, 0, "chol")
    x = np.zeros(A.n)
    for k in range(1, 5):
        x = x + lu.solve(b - A.matvec(x))
        xo, _ = ras.ordered(b, k)
        assert np.linalg.norm(xo - x) <= 1e-13 * np.linalg.norm(x)


def test_point_subdomains_are_jacobi_and_gauss_seidel():
    """One grid point per subdomain, no overlap: the synchronous sweep is the
    textbook Jacobi step and the ordered pass the Gauss-Seidel sweep in
    subdomain order, both written out component by component."""
    A = R.laplace2d(5, 4)
    S = A.scipy().tocsr()
    b = R.uniform_rhs(A.n, 9)
    owner = np.arange(A.n, dtype=np.int32)
    for loc in ("chol", "cg"):
        ras = schwarz.RAS(A, owner, 0, loc, "fp64", 2)
        xj = np.zeros(A.n)
        xg = np.zeros(A.n)
        for k in range(1, 4):
            new = np.empty(A.n)
            for i in range(A.n):
                cols, vals = S.indices[S.indptr[i]:S.indptr[i + 1]], S.data[S.indptr[i]:S.indptr[i + 1]]
                off = sum(v * xj[c] for c, v in zip(cols, vals) if c != i)
                new[i] = (b[i] - off) / S[i, i]
            xj = new
            for i in range(A.n):
                cols, vals = S.indices[S.indptr[i]:S.indptr[i + 1]], S.data[S.indptr[i]:S.indptr[i + 1]]
                off = sum(v * xg[c] for c, v in zip(cols, vals) if c != i)
                xg[i] = (b[i] - off) / S[i, i]
            xo, _, _ = ras.sync(b, 0.0, k)
            assert np.max(np.abs(xo - xj)) <= 1e-14 * np.max(np.abs(xj)), (loc, k)
            xs, _ = ras.ordered(b, k)
            assert np.max(np.abs(xs - xg)) <= 1e-14 * np.max(np.abs(xg)), (loc, k)


def test_async_simulator_converges_and_verifies():
    A = R.laplace2d(24)
    b = R.uniform_rhs(A.n, 8)
    xd = schwarz.direct_solve(A, b)
    ras = schwarz.RAS(A, partition.regular_grid(A.grid, (3, 3)), 2, "chol")
    for seed in range(3):
        x, info = ras.async_sim(b, 1e-8, seed=seed, staleness=4, max_updates=200000)
        assert info["converged"]
        assert schwarz.relative_residual(A, x, b) < 1e-8
        assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_async_simulator_decentralized_detection():
    A = R.laplace2d(24)
    b = R.uniform_rhs(A.n, 10)
    xd = schwarz.direct_solve(A, b)
    ras = schwarz.RAS(A, partition.regular_grid(A.grid, (3, 3)), 2, "chol")
    nb = ras.neighbours()
    assert sorted(nb[4].tolist()) == [0, 1, 2, 3, 5, 6, 7, 8]  # centre box reads its corners through overlap 2
    assert sorted(nb[0].tolist()) == [1, 3, 4]
    x, info = ras.async_sim(b, 1e-8, seed=3, staleness=2, max_updates=200000, detect="decentral")
    assert info["converged"] and schwarz.relative_residual(A, x, b) < 1e-8
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)


def test_async_simulator_estimate_detection():
    """The estimate detector stops on the sum of the owned residuals of every
    subdomain's latest update once all have updated; its stop is verified
    exactly, so the result meets the global criterion, and with a subdomain
    paused it cannot stop before that subdomain has updated."""
    A = R.laplace2d(24)
    b = R.uniform_rhs(A.n, 10)
    xd = schwarz.direct_solve(A, b)
    ras = schwarz.RAS(A, partition.regular_grid(A.grid, (3, 3)), 2, "chol")
    x, info = ras.async_sim(b, 1e-8, seed=3, staleness=2, max_updates=200000, detect="estimate")
    assert info["converged"] and schwarz.relative_residual(A, x, b) < 1e-8
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
    x, info = ras.async_sim(b, 1e-8, seed=3, staleness=2, max_updates=200000, detect="estimate",
                            paused={4}, pause_until=3000)
    assert info["converged"] and info["events"] > 3000 and schwarz.relative_residual(A, x, b) < 1e-8


def test_async_simulator_waits_for_paused_subdomain():
    A = R.laplace2d(16)
    b = R.uniform_rhs(A.n, 9)
    ras = schwarz.RAS(A, partition.regular_grid(A.grid, (2, 2)), 2, "chol")
    x, info = ras.async_sim(b, 1e-8, seed=1, paused={3}, pause_until=5000, max_updates=100000)
    assert info["converged"] and info["events"] > 5000


# ----------------------------------------------------------------- P11: precision variants reach tau
@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_low_precision_local_solves_reach_tolerance(storage):
    g = R.gaussian_random_field_2d(32, 4.0, 12)
    A = R.tpfa2d(np.exp(g), 10.0)
    b = R.uniform_rhs(A.n, 13)
    owner = partition.regular_grid(A.grid, (2, 2))
    ref = schwarz.RAS(A, owner, 2, "chol", "fp64").sync(b, 1e-8, 20000)
    x, hist, k = schwarz.RAS(A, owner, 2, "chol", storage).sync(b, 1e-8, 20000)
    assert hist[-1] < 1e-8
    assert np.linalg.norm(x - ref[0]) <= 1e-5 * np.linalg.norm(ref[0])


# ------------------------------------------- P12: an asynchronous update reads each value once
def _async_reads(ras, b, consistent, staleness, updates, seed):
    """Asynchronous RAS with exact local solves where every update reads other
    subdomains' values from the last `staleness` iterates: either one version per
    value for the whole update (consistent), or a version per row entry (a value
    read by several rows may be seen at different times)."""
    rng = np.random.default_rng(seed)
    M = ras.M.tocsr()
    x = np.zeros(M.shape[0])
    hist = [x]
    for _ in range(updates):
        p = int(rng.integers(ras.P))
        s = ras.subs[p]
        sub = M[s.omega]
        H = np.array(hist)
        L = len(hist)
        if consistent:
            ver = rng.integers(0, L, M.shape[0])[sub.indices]
        else:
            ver = rng.integers(0, L, sub.nnz)
        vals = H[L - 1 - ver, sub.indices]
        vals = np.where(ras.owner[sub.indices] == p, x[sub.indices], vals)
        r = b[s.omega] - np.add.reduceat(sub.data * vals, sub.indptr[:-1])
        x = x.copy()
        x[s.owned] += s.solver(r)[s.pos]
        hist = (hist + [x])[-staleness:]
    return np.linalg.norm(b - M @ x) / np.linalg.norm(b)


def test_async_update_must_read_each_value_once():
    """Reading: an asynchronous subdomain update works on one copy of the values
    it receives (Sec. 2.1), i.e. every row of its residual sees the same version
    of a neighbour's value.  With exact local solves, per-entry versions break the
    cancellation the local solve relies on and the iteration diverges under deep
    staleness, while one version per value converges (the library takes a
    snapshot per update for this reason)."""
    A = R.laplace2d(24)
    b = R.uniform_rhs(A.n, 3)
    ras = schwarz.RAS(A, partition.regular_grid(A.grid, (4, 4)), 2, "chol")
    for seed in (0, 1):
        assert _async_reads(ras, b, True, 48, 3000, seed) < 1e-5
        assert _async_reads(ras, b, False, 48, 3000, seed) > 1e3


# ----------------------------------------------------------------- timed asynchronous schedule
def _timed_case():
    A = R.laplace2d(40)
    owner = partition.rcb(A.coords(), 4, 0, 0.0)
    return A, R.uniform_rhs(A.n, 1), schwarz.RAS(A, owner, 2, "chol", "fp64")


def test_paced_lockstep_schedule_is_the_synchronous_iteration():
    """Equal update times, start times a hair apart, reads that wait for the
    neighbours: update k of every subdomain reads exactly the k-1st updates of
    its neighbours, i.e. the synchronous (Jacobi-type) sweep of Eq. 3."""
    A, b, ras = _timed_case()
    K = 12
    xs, _, _ = ras.sync(b, 0.0, K)
    xa, info = ras.async_timed(b, 0.0, np.ones(ras.P), offsets=1e-3 * np.arange(ras.P), pace=16.0, max_rounds=K)
    assert np.all(info["local_solves"] == K)
    assert np.max(np.abs(xa - xs)) <= 1e-14 * np.max(np.abs(xs))


def test_free_running_lockstep_schedule_reads_one_update_late():
    """Without the wait, a subdomain that finishes a hair before its neighbour
    reads the neighbour's update before last; evenly timed subdomains then need
    markedly more updates than synchronous sweeps, and paced reads recover the
    synchronous count up to the detection lag."""
    A, b, ras = _timed_case()
    _, _, k_sync = ras.sync(b, 1e-8, 5000)
    off = 1e-3 * np.arange(ras.P)
    _, free = ras.async_timed(b, 1e-8, np.ones(ras.P), offsets=off, pace=0.0)
    _, paced = ras.async_timed(b, 1e-8, np.ones(ras.P), offsets=off, pace=0.25)
    assert free["converged"] and paced["converged"]
    assert np.median(free["local_solves"]) >= 1.3 * k_sync
    assert np.median(paced["local_solves"]) <= k_sync + 1
