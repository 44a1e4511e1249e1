"""Property-based parity of the host setup (CPU only): on randomly drawn grids
(2-D and 3-D boxes with sides from 1, ragged against the part counts),
partitions (regular strips and boxes, seeded RCB with jitter) and overlaps, the
library's owners, overlapping sets (Sec. 2.1, Fig. 1; Sec. 3.2.1) and
communication volume (Fig. 2) equal the oracle's bit for bit; on random SPD
matrices with the grid's pattern the local factors (Sec. 3.3.1) are the
Cholesky factors of the local matrices: the band factor equals LAPACK's, the
sparse factor gives L L^T = P A_p P^T, and its solve schedules and device lane
layout give the triangular solves; FP16 row-scaled storage and ORAS (Robin)
factors follow their definitions on the same random cases."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import scipy.sparse as sp

import ras_inputs as R
from oracle import local as olocal
from oracle import overlap as oover
from oracle import partition as opart

ras = pytest.importorskip("paper_2003_05361_amd")


@st.composite
def problems(draw):
    if draw(st.booleans()):
        sides = (draw(st.integers(1, 24)), draw(st.integers(1, 24)), 1)
        A = R.laplace2d(sides[0], sides[1])
    else:
        sides = (draw(st.integers(1, 9)), draw(st.integers(1, 9)), draw(st.integers(1, 9)))
        A = R.laplace3d(*sides)
    kind = draw(st.sampled_from(["regular_1d", "regular_grid", "rcb"]))
    if kind == "regular_1d":
        P = draw(st.integers(1, min(A.n, 12)))
        part = ("regular_1d", P)
    elif kind == "regular_grid":
        parts = tuple(draw(st.integers(1, min(s, 4))) for s in sides)
        part = ("regular_2d", parts[:2]) if sides[2] == 1 else ("regular_3d", parts)
    else:
        P = draw(st.integers(1, min(A.n, 16)))
        part = ("rcb", (P, draw(st.integers(0, 2**63 - 1)), draw(st.floats(0.0, 0.9))))
    return A, part, draw(st.integers(0, 3))


@settings(max_examples=300, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(problems())
def test_index_sets_and_volume_match_the_oracle(case):
    A, (kind, arg), gamma = case
    if kind == "rcb":
        P, seed, jit = arg
        owner = opart.rcb(A.coords(), P, seed, jit)
        spec = ras.partition("rcb", P, grid=A.grid, seed=seed, jitter=jit)
    elif kind == "regular_1d":
        owner = opart.regular_1d(A.n, arg)
        spec = ras.partition("regular_1d", arg, grid=A.grid)
    else:
        owner = opart.regular_grid(A.grid, arg)
        spec = ras.partition(kind, arg, grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("cg", "fp64", 2))
    try:
        o2, ptr2, idx2 = plan.sets()
        vol = plan.comm_volume()
    finally:
        plan.close()
    sets = oover.subdomain_sets(A, owner, gamma)
    ptr, idx = oover.flatten_sets(sets)
    assert np.array_equal(o2, owner)
    assert np.array_equal(ptr2, ptr)
    assert np.array_equal(idx2, idx)
    assert np.array_equal(vol, oover.comm_volume(owner, sets))


def _random_spd(A, seed):
    """A graph Laplacian on A's pattern with weights log-uniform over four
    decades, plus a positive diagonal shift: symmetric positive definite."""
    rng = np.random.default_rng(seed)
    M = sp.csr_matrix((A.data, A.indices, A.indptr), shape=(A.n, A.n))
    U = sp.triu(M, k=1).tocoo()
    w = 10.0 ** rng.uniform(-2.0, 2.0, U.nnz)
    W = sp.coo_matrix((-w, (U.row, U.col)), shape=M.shape)
    W = (W + W.T).tocsr()
    d = -np.asarray(W.sum(axis=1)).ravel() + 10.0 ** rng.uniform(-2.0, 0.0, A.n)
    S = (W + sp.diags(d)).tocsr()
    S.sort_indices()
    return R.CSR(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.float64), A.grid)


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(problems(), st.integers(0, 2**32 - 1))
def test_local_factors_are_cholesky_factors(case, seed):
    A0, (kind, arg), gamma = case
    A = _random_spd(A0, seed)
    if kind == "rcb":
        spec = ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2])
    else:
        spec = ras.partition(kind, arg, grid=A.grid)
    band_plan = ras.Plan(A, spec, gamma, ras.local("chol", "fp64"))
    sparse_plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", "fp64"))
    try:
        _, ptr, idx = band_plan.sets()
        for p in range(len(ptr) - 1):
            om = idx[ptr[p]:ptr[p + 1]]
            n = om.size
            Ap = olocal.local_matrix(A, om)
            # band factor against LAPACK's banded Cholesky of the same local matrix
            band, w = band_plan.factor(p)
            cb, w_ref = olocal.band_cholesky(Ap)
            # the stored width is at least 1: a diagonal local matrix keeps one
            # zero sub-diagonal (LAPACK's band form has width 0 there)
            assert w == max(w_ref, 1)
            if w_ref == 0:
                assert np.all(band[:, 0] == 0.0)
            L_ref = olocal.band_to_dense_lower(cb)
            L = np.zeros((n, n))
            for o in range(w + 1):
                i = np.arange(n)
                j = i - w + o
                m = j >= 0
                L[i[m], j[m]] = band[i[m], o]
            assert np.max(np.abs(L - L_ref)) <= 1e-12 * np.max(np.abs(L_ref))
            # sparse factor: a permutation and a lower-triangular L with L L^T = P A_p P^T
            perm, rp, col, val, diag = sparse_plan.sparse_factor(p)
            assert np.array_equal(np.sort(perm), np.arange(n)) and np.all(diag > 0)
            Ls = np.zeros((n, n))
            for k in range(n):
                cs = col[rp[k]:rp[k + 1]]
                assert np.all(cs < k) and np.all(np.diff(cs) > 0)
                Ls[k, cs] = val[rp[k]:rp[k + 1]]
                Ls[k, k] = diag[k]
            Ad = Ap.toarray()[np.ix_(perm, perm)]
            assert np.max(np.abs(Ls @ Ls.T - Ad)) <= 1e-12 * np.max(np.abs(Ad))
    finally:
        band_plan.close()
        sparse_plan.close()


@settings(max_examples=100, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(problems(), st.integers(0, 2**32 - 1), st.sampled_from(["fp64", "fp32"]))
def test_sparse_schedules_and_lanes_solve_the_triangular_systems(case, seed, storage):
    """Both passes of every subdomain's solve schedule, and the lane layout the
    device streams, run with parallel step semantics (race-free, checked by the
    simulators), give L^{-1} v and L^{-T} v to rounding."""
    import scipy.sparse.linalg as spla

    from test_host_parity import _run_lanes, _run_schedule

    A0, (kind, arg), gamma = case
    A = _random_spd(A0, seed)
    if kind == "rcb":
        spec = ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2])
    else:
        spec = ras.partition(kind, arg, grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", storage))
    rng = np.random.default_rng(seed)
    try:
        _, ptr, _ = plan.sets()
        for p in range(len(ptr) - 1):
            n = int(ptr[p + 1] - ptr[p])
            perm, rp, col, val, diag = plan.sparse_factor(p)
            L = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
            v = rng.standard_normal(n)
            for pass_, M, lower in ((0, L, True), (1, L.T.tocsr(), False)):
                ref = spla.spsolve_triangular(M, v, lower=lower)
                scale = max(np.max(np.abs(ref)), 1e-300)
                sch = plan.sparse_schedule(p, pass_)
                assert np.max(np.abs(_run_schedule(sch, v) - ref)) <= 1e-11 * scale, (p, pass_)
                lay = plan.sparse_lanes(p, pass_)
                assert np.max(np.abs(_run_lanes(lay, v, sch["slots"]) - ref)) <= 1e-11 * scale, (p, pass_)
    finally:
        plan.close()


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(problems(), st.integers(0, 2**32 - 1))
def test_fp16_rowscaled_storage_quantises_the_band_factor(case, seed):
    """FP16_ROWSCALED storage of every subdomain's factor: scale[i] =
    float32(max_j |L_ij|) (1 for a zero row) and each stored slot the float16
    (round to nearest even from float64) of L_ij / scale[i], bit for bit against
    numpy's conversion of the library's own float64 factor."""
    A0, (kind, arg), gamma = case
    A = _random_spd(A0, seed)
    if kind == "rcb":
        spec = ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2])
    else:
        spec = ras.partition(kind, arg, grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("chol", "fp16"))
    try:
        _, ptr, _ = plan.sets()
        for p in range(len(ptr) - 1):
            band, w = plan.factor(p)
            bits, scale = plan.factor_fp16(p)
            mx = np.max(np.abs(band), axis=1)
            ref_scale = np.where(mx > 0, mx, 1.0).astype(np.float32)
            assert np.array_equal(scale, ref_scale), p
            ref_bits = (band / scale.astype(np.float64)[:, None]).astype(np.float16).view(np.uint16)
            assert np.array_equal(bits, ref_bits), p
    finally:
        plan.close()


@settings(max_examples=60, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(problems(), st.integers(0, 2**32 - 1), st.floats(0.05, 1.0))
def test_oras_factors_are_cholesky_of_the_robin_local_matrices(case, seed, q):
    """ORAS plans (a Robin transmission condition in algebraic form): the band
    and the sparse factor of every subdomain are Cholesky factors of the oracle's
    Robin local matrix, A[Omega_p, Omega_p] with the diagonal lowered by
    (1 - q) times the coupling to points outside Omega_p."""
    A0, (kind, arg), gamma = case
    A = _random_spd(A0, seed)
    if kind == "rcb":
        spec = ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2])
    else:
        spec = ras.partition(kind, arg, grid=A.grid)
    band_plan = ras.Plan(A, spec, gamma, ras.local("chol", "fp64", robin_q=q))
    sparse_plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", "fp64", robin_q=q))
    try:
        _, ptr, idx = band_plan.sets()
        for p in range(len(ptr) - 1):
            om = idx[ptr[p]:ptr[p + 1]]
            n = om.size
            Ar = olocal.robin_local_matrix(A, om, q).toarray()
            band, w = band_plan.factor(p)
            L = np.zeros((n, n))
            for o in range(w + 1):
                i = np.arange(n)
                j = i - w + o
                m = j >= 0
                L[i[m], j[m]] = band[i[m], o]
            assert np.max(np.abs(L @ L.T - Ar)) <= 1e-12 * np.max(np.abs(Ar)), p
            perm, rp, col, val, diag = sparse_plan.sparse_factor(p)
            Ls = np.zeros((n, n))
            for k in range(n):
                Ls[k, col[rp[k]:rp[k + 1]]] = val[rp[k]:rp[k + 1]]
                Ls[k, k] = diag[k]
            Ad = Ar[np.ix_(perm, perm)]
            assert np.max(np.abs(Ls @ Ls.T - Ad)) <= 1e-12 * np.max(np.abs(Ad)), p
    finally:
        band_plan.close()
        sparse_plan.close()
