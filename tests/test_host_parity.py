"""Host-side setup of the native library vs the oracle (CPU only, no GPU calls).

Index sets must match bit-exactly; factors to rounding; FP16 quantisation
bit-exactly; invalid inputs must come back as error codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import ras_inputs as R
from oracle import local as olocal
from oracle import overlap as oover
from oracle import partition as opart

ras = pytest.importorskip("paper_2003_05361_amd")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(ras.LIB_PATH):
        pytest.skip("native library not built")
    return ras.lib()


def test_header_symbols_exported():
    lib = _lib_or_skip()
    header = open(os.path.join(ROOT, "include", "ras.h")).read()
    declared = set(re.findall(r"\b(ras_[a-z0-9_]+)\s*\(", header))
    declared -= {"ras_status"}
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(ras.SIGNATURES), declared ^ set(ras.SIGNATURES)


def test_null_arguments_are_argument_errors():
    """Every entry point that takes a plan, handle or server, or output pointers,
    answers NULL with RAS_E_ARG (-1) before touching a device; destroying NULL
    is a no-op."""
    lib = _lib_or_skip()
    calls = {
        "ras_plan_create": lambda: lib.ras_plan_create(None, None, 1, None, None),
        "ras_plan_get_stats": lambda: lib.ras_plan_get_stats(None, None),
        "ras_plan_sets": lambda: lib.ras_plan_sets(None, None, None, None),
        "ras_plan_factor": lambda: lib.ras_plan_factor(None, 0, None, None),
        "ras_plan_factor_fp16": lambda: lib.ras_plan_factor_fp16(None, 0, None, None),
        "ras_plan_sparse_factor": lambda: lib.ras_plan_sparse_factor(None, 0, None, None, None, None, None, None),
        "ras_plan_sparse_schedule": lambda: lib.ras_plan_sparse_schedule(None, 0, 0, None, None, None, None, None,
                                                                         None, None, None, None),
        "ras_plan_sparse_lanes": lambda: lib.ras_plan_sparse_lanes(None, 0, 0, None, None, None, None, None),
        "ras_setup": lambda: lib.ras_setup(None, None, 1, None, None, None),
        "ras_setup_from_plan": lambda: lib.ras_setup_from_plan(None, None, None),
        "ras_pause": lambda: lib.ras_pause(None, 0, 1),
        "ras_cancel": lambda: lib.ras_cancel(None),
        "ras_handle_get_stats": lambda: lib.ras_handle_get_stats(None, None),
        "ras_solve": lambda: lib.ras_solve(None, None, None, 1, None, None),
        "ras_solve_noalloc": lambda: lib.ras_solve_noalloc(None, None, None, 1, None, None),
        "ras_batch_solve": lambda: lib.ras_batch_solve(0, None, None, None, None, None, None),
        "ras_residual_history": lambda: lib.ras_residual_history(None, 0, None, None, 0, None),
        "ras_local_solve_counts": lambda: lib.ras_local_solve_counts(None, 0, None),
        "ras_partition_sets": lambda: lib.ras_partition_sets(None, None, None, None),
        "ras_phase_seconds": lambda: lib.ras_phase_seconds(None, 0, None),
        "ras_autotune": lambda: lib.ras_autotune(None, None, None, 1, None, None),
        "ras_handle_factor": lambda: lib.ras_handle_factor(None, 0, None, None),
        "ras_relative_residual": lambda: lib.ras_relative_residual(None, None, None, None),
        "ras_server_create": lambda: lib.ras_server_create(0, 0.01, None, None),
        "ras_server_submit": lambda: lib.ras_server_submit(None, None, None, 1, None, None, 1, 1e-8, None),
        "ras_server_poll": lambda: lib.ras_server_poll(None, 0, None, None, None),
        "ras_server_wait": lambda: lib.ras_server_wait(None, 0, 0.0),
        "ras_server_get_stats": lambda: lib.ras_server_get_stats(None, None),
    }
    for name, call in calls.items():
        assert call() == -1, name
        assert lib.ras_last_error(), name
    assert lib.ras_server_destroy(None) == 0
    lib.ras_destroy(None)
    lib.ras_plan_destroy(None)


def _oracle_sets(A, owner, gamma):
    sets = oover.subdomain_sets(A, owner, gamma)
    return oover.flatten_sets(sets)


CASES = [
    ("poisson2d_64_strips4", R.laplace2d(64), ("regular_1d", 4), 2),
    ("poisson2d_96_3x4", R.laplace2d(96, 80), ("regular_2d", (3, 4)), 4),
    ("laplace3d_20_rcb16", R.laplace3d(20), ("rcb", (16, 3, 0.4)), 1),
    ("laplace3d_18_2x3x2", R.laplace3d(18), ("regular_3d", (2, 3, 2)), 2),
    ("laplace2d_33_rcb7_g0", R.laplace2d(33, 17), ("rcb", (7, 11, 0.3)), 0),
    # ragged: grid sides that the part counts do not divide
    ("laplace2d_37x23_4x3_g2", R.laplace2d(37, 23), ("regular_2d", (4, 3)), 2),
    ("laplace2d_37x23_strips7_g3", R.laplace2d(37, 23), ("regular_1d", 7), 3),
    ("laplace3d_13x11x7_4x3x2_g2", R.laplace3d(13, 11, 7), ("regular_3d", (4, 3, 2)), 2),
]


@pytest.mark.parametrize("name,A,part,gamma", CASES, ids=[c[0] for c in CASES])
def test_index_sets_bit_exact(name, A, part, gamma):
    _lib_or_skip()
    kind, arg = part
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
    plan = ras.Plan(A, spec, gamma, ras.local("cg", "fp64", 3))
    o2, ptr2, idx2 = plan.sets()
    ptr, idx = _oracle_sets(A, owner, gamma)
    assert np.array_equal(o2, owner)
    assert np.array_equal(ptr2, ptr)
    assert np.array_equal(idx2, idx)


# the three full-size workloads, in the partitions and overlaps they are solved with
FULL_SIZE = [
    ("poisson2d_1024_8x8_g4", lambda: R.laplace2d(1024), ("regular_2d", (8, 8)), 4),
    ("laplace3d_128_rcb256_g1", lambda: R.laplace3d(128), ("rcb", (256, 3, 0.4)), 1),
    ("diffusion2d_2048_16x16_g4", lambda: R.config_problem("diffusion2d_2048_16x16")[0], ("regular_2d", (16, 16)), 4),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,make,part,gamma", FULL_SIZE, ids=[c[0] for c in FULL_SIZE])
def test_index_sets_bit_exact_full_size(name, make, part, gamma):
    """owner, omega_ptr and omega_idx of the full-size workloads, bit-exact against
    the oracle's partition and breadth-first overlap."""
    _lib_or_skip()
    A = make()
    kind, arg = part
    if kind == "rcb":
        P, seed, jit = arg
        owner = opart.rcb(A.coords(), P, seed, jit)
        spec = ras.partition("rcb", P, grid=A.grid, seed=seed, jitter=jit)
    else:
        owner = opart.regular_grid(A.grid, arg)
        spec = ras.partition(kind, arg, grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("cg", "fp64", 1))
    o2, ptr2, idx2 = plan.sets()
    plan.close()
    assert np.array_equal(o2, owner)
    ptr, idx = _oracle_sets(A, owner, gamma)
    assert ptr2.dtype == np.int64 and idx2.dtype == np.int32
    assert np.array_equal(ptr2, ptr)
    assert np.array_equal(idx2, idx)


@pytest.mark.parametrize("name,A,part,gamma", CASES, ids=[c[0] for c in CASES])
def test_comm_volume_bit_exact(name, A, part, gamma):
    _lib_or_skip()
    kind, arg = part
    if kind == "rcb":
        spec = ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2])
    else:
        spec = ras.partition(kind, arg, grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("cg", "fp64", 3))
    owner, _, _ = plan.sets()
    vol = plan.comm_volume()
    ref = oover.comm_volume(owner, oover.subdomain_sets(A, owner, gamma))
    assert vol.dtype == np.int64 and np.array_equal(vol, ref)


def test_comm_volume_single_subdomain():
    _lib_or_skip()
    A = R.laplace2d(9)
    plan = ras.Plan(A, ras.partition("regular_1d", 1, grid=A.grid), 3, ras.local("chol", "fp64"))
    assert np.array_equal(plan.comm_volume(), np.zeros((1, 1), dtype=np.int64))
    lib = ras.lib()
    assert lib.ras_plan_comm_volume(plan._p, None) == -1
    assert lib.ras_plan_comm_volume(None, np.zeros(1, np.int64).ctypes.data) == -1


def test_rcb_config3_partition_bit_exact():
    """The 128^3, 256-part, jitter 0.4 partition of the 3-D workload."""
    _lib_or_skip()
    A = R.laplace3d(128)
    owner = opart.rcb(A.coords(), 256, 3, 0.4)
    plan = ras.Plan(A, ras.partition("rcb", 256, grid=A.grid, seed=3, jitter=0.4), 0, ras.local("cg", "fp32", 8))
    o2, _, _ = plan.sets()
    assert np.array_equal(o2, owner)
    counts = np.bincount(owner)
    assert counts.min() >= 0.5 * A.n / 256 and counts.max() <= 1.5 * A.n / 256


def test_band_factor_matches_lapack():
    _lib_or_skip()
    g = R.gaussian_random_field_2d(40, 6.0, 21)
    A = R.tpfa2d(np.exp(2 * g), 10.0)
    owner = opart.regular_grid(A.grid, (2, 2))
    plan = ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 3, ras.local("chol", "fp64"))
    sets = oover.subdomain_sets(A, owner, 3)
    for p, (_, om, _) in enumerate(sets):
        band, w = plan.factor(p)
        Ap = olocal.local_matrix(A, om)
        cb, w_ref = olocal.band_cholesky(Ap)
        assert w == w_ref
        n = om.size
        # oracle lower band form cb[k, j] = L[j+k, j]  <->  row-major band[i, o] = L[i, i-w+o]
        L_ref = olocal.band_to_dense_lower(cb)
        L = np.zeros((n, n))
        for o in range(w + 1):
            i = np.arange(n)
            j = i - w + o
            m = j >= 0
            L[i[m], j[m]] = band[i[m], o]
        assert np.max(np.abs(L - L_ref)) <= 1e-13 * np.max(np.abs(L_ref))


def test_fp16_rowscaled_quantisation_bit_exact():
    _lib_or_skip()
    g = R.gaussian_random_field_2d(24, 4.0, 5)
    A = R.tpfa2d(np.exp(2 * g), 10.0)
    owner = opart.regular_grid(A.grid, (2, 1))
    plan = ras.Plan(A, ras.partition("regular_2d", (2, 1), grid=A.grid), 2, ras.local("chol", "fp16"))
    sets = oover.subdomain_sets(A, owner, 2)
    for p, (_, om, _) in enumerate(sets):
        bits, scale = plan.factor_fp16(p)
        band, w = plan.factor(p)
        Ap = olocal.local_matrix(A, om)
        cb, _ = olocal.band_cholesky(Ap)
        Lhat, s = olocal.quantize_rows_fp16(cb)
        n = om.size
        assert np.array_equal(scale, s)
        # compare every stored band slot: row-major (i, o) <-> lapack (k = w - o, j = i - w + o)
        for o in range(w + 1):
            i = np.arange(n)
            j = i - w + o
            m = j >= 0
            ours = bits[i[m], o]
            ref = Lhat[w - o, j[m]].view(np.uint16)
            # the oracle quantises from its own LAPACK factor: equal up to the rare
            # case where the two FP64 factors differ in the last bit across a tie
            assert np.mean(ours == ref) > 0.999
            assert np.all(np.abs(ours.view(np.float16).astype(np.float64) - ref.view(np.float16).astype(np.float64))
                          <= 2.0 ** -10)


def test_fp16_conversion_rounding_matches_numpy():
    """The host's float64 -> float16 rounding agrees with numpy's (round to nearest even)."""
    _lib_or_skip()
    # build a one-subdomain diagonal system whose factor entries are chosen values
    vals = np.array([1.0, 1 + 2**-11, 1 + 3 * 2**-11, 0.5 + 2**-12, 2.0**-20, 2.0**-25, 2.0**-24 * 1.5,
                     0.999755859375, 0.9997558593750001, 1e-8, 3.0**-1])
    diag = vals**2
    A = sp.diags(diag).tocsr()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    plan = ras.Plan(A, ras.partition("explicit", 1, owner=np.zeros(len(diag), np.int32)), 0,
                    ras.local("chol", "fp16"))
    bits, scale = plan.factor_fp16(0)
    band, w = plan.factor(0)
    # a diagonal matrix is stored with one zero sub-diagonal
    assert w == 1 and np.all(band[:, 0] == 0) and np.all(bits[:, 0] == 0)
    assert np.array_equal(band[:, 1], vals)
    ref = (band[:, 1] / scale.astype(np.float64)).astype(np.float16).view(np.uint16)
    assert np.array_equal(bits[:, 1], ref)
    # direct conversion checks through a 2-entry row: L = [[a,0],[b,c]] -> row scale max(|b|,|c|)
    A2 = sp.csr_matrix(np.array([[1.0, 2.0**-12], [2.0**-12, 1.0]]))
    A2.indptr = A2.indptr.astype(np.int64)
    A2.indices = A2.indices.astype(np.int32)
    plan2 = ras.Plan(A2, ras.partition("explicit", 1, owner=np.zeros(2, np.int32)), 0, ras.local("chol", "fp16"))
    b2, s2 = plan2.factor_fp16(0)
    f2, _ = plan2.factor(0)
    assert np.array_equal(b2, (f2 / s2.astype(np.float64)[:, None]).astype(np.float16).view(np.uint16))


@pytest.mark.parametrize("bad", ["unsorted", "duplicate", "range", "unsym", "rowptr"])
def test_invalid_csr_rejected(bad):
    _lib_or_skip()
    A = R.laplace2d(4).scipy().tocsr()
    indptr = A.indptr.astype(np.int64).copy()
    indices = A.indices.astype(np.int32).copy()
    data = A.data.copy()
    if bad == "unsorted":
        indices[0], indices[1] = indices[1], indices[0]
    elif bad == "duplicate":
        indices[1] = indices[0]
    elif bad == "range":
        indices[-1] = 99
    elif bad == "unsym":
        M = A.tolil()
        M[0, 15] = -0.5
        M = M.tocsr()
        indptr, indices, data = M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data
    elif bad == "rowptr":
        indptr[3] = indptr[2] - 1

    class Fake:
        pass

    F = Fake()
    F.indptr, F.indices, F.data, F.grid = indptr, indices, data, (4, 4, 1)
    with pytest.raises(ras.RasError) as e:
        ras.Plan(F, ras.partition("regular_1d", 2), 1, ras.local("cg", "fp64", 2))
    assert e.value.status == -2


def test_invalid_arguments_rejected():
    _lib_or_skip()
    A = R.laplace2d(8)
    cases = [
        (ras.partition("regular_1d", 0), 1, ras.local("cg", "fp64", 2)),
        (ras.partition("regular_1d", 65), 1, ras.local("cg", "fp64", 2)),
        (ras.partition("regular_2d", (2, 2), grid=(8, 7, 1)), 1, ras.local("cg", "fp64", 2)),
        (ras.partition("regular_1d", 2), -1, ras.local("cg", "fp64", 2)),
        (ras.partition("regular_1d", 2), 1, ras.local("cg", "fp64", 0)),
        (ras.partition("regular_1d", 2), 1, ras.local("cg", "fp16", 2)),
        (ras.partition("explicit", 3, owner=np.zeros(64, np.int32)), 1, ras.local("cg", "fp64", 2)),
        (ras.partition("rcb", 4, grid=A.grid, jitter=1.5), 1, ras.local("cg", "fp64", 2)),
    ]
    for part, gamma, loc in cases:
        with pytest.raises(ras.RasError) as e:
            ras.Plan(A, part, gamma, loc)
        assert e.value.status == -1, (part, gamma, loc)


def test_not_spd_reported():
    _lib_or_skip()
    A = R.laplace2d(6).scipy().tolil()
    A[7, 7] = -4.0
    A = A.tocsr()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    with pytest.raises(ras.RasError) as e:
        ras.Plan(A, ras.partition("regular_1d", 2), 1, ras.local("chol", "fp64"))
    assert e.value.status == -3
    assert "subdomain 0" in str(e.value)


def test_plan_stats_config2_shape():
    """1024^2 grid, 8x8 boxes, overlap 4: local sizes between 17,414 and 18,456 rows."""
    _lib_or_skip()
    A = R.laplace2d(1024)
    plan = ras.Plan(A, ras.partition("regular_2d", (8, 8), grid=A.grid), 4, ras.local("cg", "fp64", 10))
    st = plan.stats()
    assert st["parts"] == 64 and st["max_ell_width"] == 5
    assert st["min_local_rows"] == 17414 and st["max_local_rows"] == 18456


# ----------------------------------------------------------------------------- sparse Cholesky (host)
SPARSE_CASES = [
    # degenerate: one unknown, and a 1-D chain whose separators are single points
    ("one_unknown", R.CSR(np.array([0, 1], np.int64), np.array([0], np.int32), np.array([4.0]), (1, 1, 1)),
     ("regular_1d", 1), 0),
    ("chain_16_halves_g1", R.laplace2d(16, 1), ("regular_1d", 2), 1),
    ("poisson2d_40_2x2_g3", R.laplace2d(40), ("regular_2d", (2, 2)), 3),
    ("laplace3d_12_rcb5_g1", R.laplace3d(12), ("rcb", (5, 2, 0.3)), 1),
    ("tpfa2d_24_strips3_g2", R.tpfa2d(np.exp(2 * R.gaussian_random_field_2d(24, 4.0, 3)), 10.0), ("regular_1d", 3), 2),
]


@pytest.mark.parametrize("name,A,part,gamma", SPARSE_CASES, ids=[c[0] for c in SPARSE_CASES])
def test_sparse_factor_is_cholesky_of_permuted_local_matrix(name, A, part, gamma):
    """L L^T = A_p[perm][:, perm] with L lower triangular and a positive diagonal,
    perm a permutation of the local rows (Sec. 3.3.1: exact local solves)."""
    _lib_or_skip()
    kind, arg = part
    spec = (ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2]) if kind == "rcb"
            else ras.partition(kind, arg, grid=A.grid))
    plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", "fp64"))
    owner, ptr, idx = plan.sets()
    M = A.scipy().tocsr()
    for p in range(len(ptr) - 1):
        om = idx[ptr[p]:ptr[p + 1]]
        n = om.size
        perm, rp, col, val, diag = plan.sparse_factor(p)
        assert np.array_equal(np.sort(perm), np.arange(n))
        assert np.all(diag > 0)
        L = np.zeros((n, n))
        for k in range(n):
            cs = col[rp[k]:rp[k + 1]]
            assert np.all(cs < k) and np.all(np.diff(cs) > 0)
            L[k, cs] = val[rp[k]:rp[k + 1]]
            L[k, k] = diag[k]
        Ap = M[om][:, om].toarray()[np.ix_(perm, perm)]
        assert np.max(np.abs(L @ L.T - Ap)) <= 1e-12 * np.max(np.abs(Ap))


def _run_schedule(sch, v):
    """Applies a solve schedule step by step with parallel semantics (every record
    of a step reads the values as they were before the step) and checks that it
    is race-free: no two records of a step write one slot, no record reads a
    slot written in its own step, block slots are written before they are read."""
    n = v.size
    y = np.concatenate([v, np.full(sch["slots"], np.nan)])
    written = np.full(y.size, -1)
    sp_, meta, col, val = sch["step_ptr"], sch["meta"], sch["col"], sch["val"]
    assert sp_[0] == 0 and sp_[-1] == len(meta) and np.all(np.diff(sp_) > 0)
    assert np.all(meta[:, 3] == 0) and np.all(meta[:-1, 2] == meta[1:, 1])
    for s in range(len(sp_) - 1):
        recs = meta[sp_[s]:sp_[s + 1]]
        dest = recs[:, 0]
        assert np.unique(dest).size == dest.size
        in_step = np.zeros(y.size, dtype=bool)
        in_step[dest] = True
        new = np.empty(len(recs))
        for r, (d, e0, e1, _) in enumerate(recs):
            cs = col[e0:e1]
            # a record may read its own row's initial value (the right-hand side)
            assert not np.any(in_step[cs] & (cs != d)), (s, d)
            assert np.all(written[cs[cs >= n]] >= 0)
            assert not np.any((cs == d) & (written[cs] >= 0))
            new[r] = np.dot(val[e0:e1], y[cs])
        y[dest] = new
        written[dest] = s
    assert np.all(written[:n] >= 0)
    return y[:n]


def _levels(rp, col, n, forward):
    """Levels of the plain level-scheduled pass: longest dependency chains."""
    lev = np.zeros(n, dtype=np.int64)
    if forward:
        for k in range(n):
            cs = col[rp[k]:rp[k + 1]]
            lev[k] = lev[cs].max() + 1 if cs.size else 0
    else:
        deps = [[] for _ in range(n)]
        for k in range(n):
            for j in col[rp[k]:rp[k + 1]]:
                deps[j].append(k)
        for k in range(n - 1, -1, -1):
            lev[k] = max((lev[i] for i in deps[k]), default=-1) + 1
    return int(lev.max()) + 1


@pytest.mark.parametrize("name,A,part,gamma", SPARSE_CASES, ids=[c[0] for c in SPARSE_CASES])
@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_sparse_schedule_solves_the_triangular_systems(name, A, part, gamma, storage):
    """Both passes of every subdomain's solve schedule (level scheduling with dense
    diagonal blocks solved through their explicit inverses), applied in float64
    with parallel step semantics, are race-free and give L^{-1} v and L^{-T} v
    to rounding (scipy's triangular solves)."""
    _lib_or_skip()
    kind, arg = part
    spec = (ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2]) if kind == "rcb"
            else ras.partition(kind, arg, grid=A.grid))
    plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", storage))
    _, ptr, _ = plan.sets()
    rng = np.random.default_rng(11)
    import scipy.sparse.linalg as spla
    for p in range(len(ptr) - 1):
        n = int(ptr[p + 1] - ptr[p])
        perm, rp, col, val, diag = plan.sparse_factor(p)
        L = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
        v = rng.standard_normal(n)
        for pass_, M, lower in ((0, L, True), (1, L.T.tocsr(), False)):
            sch = plan.sparse_schedule(p, pass_)
            y = _run_schedule(sch, v)
            ref = spla.spsolve_triangular(M, v, lower=lower)
            assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref)), (p, pass_)
            assert len(sch["step_ptr"]) - 1 <= _levels(rp, col, n, pass_ == 0)


def _run_lanes(lay, v, nslots):
    """Applies a pass in the device's lane layout with the kernel's semantics:
    every wave streams its rounds, a lane adds val * y[col] to its sum, a
    terminator (column 0xfffe) in every lane of a group of 2^g lanes has the
    group add its sums and write the total to the slot held with g in the low
    32 bits of the value, a marker round (column 0xffff) ends the wave's part
    of a step and all waves meet there.  Within a step the waves and lanes run
    in any order; here each step is applied wave by wave with the values of
    the step's start for reads, and a read of a slot written in the same step
    fails.  Padding items (0, 0) add nothing and are exempt."""
    n = v.size
    y = np.concatenate([v, np.full(nslots, np.nan)])
    wave, col, val = lay["wave"], lay["col"], lay["val"]
    TERM, MARK = 0xFFFE, 0xFFFF
    pay_all = val.view(np.uint64) & np.uint64(0xFFFFFFFF)
    streams = []
    for w0, nr in wave:
        c = col[w0:w0 + nr]
        marks = np.flatnonzero(np.all(c == MARK, axis=1))
        assert not np.any(c[np.setdiff1d(np.arange(nr), marks)] == MARK)
        streams.append((c, val[w0:w0 + nr], pay_all[w0:w0 + nr], np.concatenate([[-1], marks])))
    nsteps = {len(m) - 1 for _, _, _, m in streams}
    assert len(nsteps) == 1  # every wave meets every barrier
    lanes = np.arange(64)
    for s in range(nsteps.pop()):
        start = y.copy()
        wrote = np.zeros(y.size, dtype=bool)
        for c, vv, pay, marks in streams:
            acc = np.zeros(64)
            g = None
            for r in range(marks[s] + 1, marks[s + 1]):
                cr, vr = c[r], vv[r]
                term = cr == TERM
                pad = (cr == 0) & (vr == 0)
                rd = ~term & ~pad
                assert not np.any(wrote[cr[rd]]), s
                acc[rd] += vr[rd] * start[cr[rd]]
                if term.any():
                    pr = pay[r][term].astype(np.int64)
                    gr = (pr >> 24) & 7
                    g = gr[0] if g is None else g
                    assert np.all(gr == g)  # one group width per wave and step
                    G = 1 << int(g)
                    dest = np.zeros(64, dtype=np.int64)
                    dest[term] = pr & 0xFFFFFF
                    tg = term.reshape(-1, G)
                    assert np.all(tg.all(axis=1) | ~tg.any(axis=1))  # whole groups end together
                    dg = dest.reshape(-1, G)[tg.any(axis=1)]
                    assert np.all(dg.min(axis=1) == dg.max(axis=1))
                    sums = acc.reshape(-1, G).sum(axis=1)
                    lead = term & (lanes % G == 0)
                    assert not np.any(wrote[dest[lead]])
                    y[dest[lead]] = sums[lanes[lead] // G]
                    wrote[dest[lead]] = True
                    acc[term] = 0.0
    return y[:n]


@pytest.mark.parametrize("name,A,part,gamma", SPARSE_CASES, ids=[c[0] for c in SPARSE_CASES])
def test_sparse_lane_layout_applies_the_schedule(name, A, part, gamma):
    """The device layout of both passes, run with the kernel's semantics, gives
    the triangular solves, every slot written once per step, no read of a value
    written in the same step, and bounded padding."""
    _lib_or_skip()
    kind, arg = part
    spec = (ras.partition("rcb", arg[0], grid=A.grid, seed=arg[1], jitter=arg[2]) if kind == "rcb"
            else ras.partition(kind, arg, grid=A.grid))
    plan = ras.Plan(A, spec, gamma, ras.local("chol_sparse", "fp64"))
    _, ptr, _ = plan.sets()
    rng = np.random.default_rng(12)
    import scipy.sparse.linalg as spla
    for p in range(len(ptr) - 1):
        n = int(ptr[p + 1] - ptr[p])
        perm, rp, col, val, diag = plan.sparse_factor(p)
        L = (sp.csr_matrix((val, col, rp), shape=(n, n)) + sp.diags(diag)).tocsr()
        v = rng.standard_normal(n)
        for pass_, M, lower in ((0, L, True), (1, L.T.tocsr(), False)):
            sch = plan.sparse_schedule(p, pass_)
            lay = plan.sparse_lanes(p, pass_)
            # the waves tile the stream, each a whole number of 8-round load groups
            # (the device loads a group ahead without checking a wave's end)
            w0, nr = lay["wave"][:, 0], lay["wave"][:, 1]
            assert np.all(nr > 0) and np.all(nr % 8 == 0), (p, pass_, nr)
            assert w0[0] == 0 and np.array_equal(w0[1:], np.cumsum(nr)[:-1]) and nr.sum() == lay["col"].shape[0]
            y = _run_lanes(lay, v, sch["slots"])
            ref = spla.spsolve_triangular(M, v, lower=lower)
            assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref)), (p, pass_)
            # the longest wave is no longer than one record per lane would make it,
            # rounded up to a whole load group
            meta = sch["meta"]
            longest = sum(int((meta[a:b, 2] - meta[a:b, 1]).max()) + 2
                          for a, b in zip(sch["step_ptr"][:-1], sch["step_ptr"][1:]))
            assert lay["wave"][:, 1].max() <= -(-longest // 8) * 8, p


def test_sparse_schedule_cuts_the_steps_of_a_grid_box():
    """An interior 136^2 box (128^2 owned, overlap 4) of a 2-D grid: the plain
    level schedule has hundreds of levels per pass (the separators are dense
    chains); with the separators' blocks solved through their inverses the
    passes take at least 4x fewer steps, in both storages, and the device
    layout spreads them evenly over the workgroup's lanes."""
    _lib_or_skip()
    A = R.laplace2d(384)
    for storage, most in (("fp64", 60), ("fp32", 45)):
        plan = ras.Plan(A, ras.partition("regular_2d", (3, 3), grid=A.grid), 4, ras.local("chol_sparse", storage))
        p = 4  # the interior box
        perm, rp, col, val, diag = plan.sparse_factor(p)
        n = perm.size
        assert n == 136 * 136 - 4 * 10
        for pass_ in (0, 1):
            sch = plan.sparse_schedule(p, pass_)
            steps = len(sch["step_ptr"]) - 1
            assert steps <= most and 4 * steps <= _levels(rp, col, n, pass_ == 0), (storage, pass_, steps)
            assert sch["min_block"] > 0 and (n + sch["slots"]) * (8 if storage == "fp64" else 4) <= 160 * 1024 - 4096
            # device layout: padding under 25 % of the items, the longest wave within
            # 1.4x of the items spread evenly over the workgroup's lanes
            lay = plan.sparse_lanes(p, pass_)
            items = len(sch["col"]) + len(sch["meta"])
            rounds = lay["wave"][:, 1]
            assert rounds.sum() * 64 <= 1.25 * items
            assert rounds.max() <= 1.4 * items / (64 * len(rounds))


def test_nested_dissection_reduces_fill_of_wide_bands():
    """A strip of 8 grid lines of a 96-wide grid: the natural order's band is the
    grid width, nested dissection keeps the factor several times smaller."""
    _lib_or_skip()
    A = R.laplace2d(96, 32)
    plan = ras.Plan(A, ras.partition("regular_1d", 4, grid=A.grid), 0, ras.local("chol_sparse", "fp64"))
    _, ptr, _ = plan.sets()
    for p in range(4):
        n = int(ptr[p + 1] - ptr[p])
        _, rp, _, _, _ = plan.sparse_factor(p)
        band_entries = n * (plan.band_width(p) + 1)
        assert rp[-1] + n < 0.5 * band_entries, (rp[-1], band_entries)


def test_sparse_solver_arguments():
    _lib_or_skip()
    A = R.laplace2d(12)
    with pytest.raises(ras.RasError) as e:
        ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol_sparse", "fp16"))
    assert e.value.status == -1
    assert ras.sparse_max_rows("fp64") > 18000 and ras.sparse_max_rows("fp32") == 2 * ras.sparse_max_rows("fp64")
    assert ras.sparse_max_rows("fp16") == 0
    plan = ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol", "fp64"))
    with pytest.raises(ras.RasError) as e:
        plan.sparse_factor(0)
    assert e.value.status == -6


def test_sparse_solver_lds_capacity():
    """The sparse solve keeps a subdomain's vector and its block slots in one
    workgroup's LDS. A 3-D box with more rows than fit is rejected at set-up in
    FP64 (E_UNSUPPORTED) and accepted in FP32 (half the bytes per value); at the
    largest boxes that fit, no dense block has room and the schedule keeps plain
    levels (min_block 0, no slots)."""
    _lib_or_skip()
    cap = {st: ras.sparse_max_rows(st) for st in ("fp64", "fp32")}
    # (box side, storage, fits, no room left for a dense block)
    for N, storage, fits, full in ((30, "fp64", False, False), (30, "fp32", True, False),
                                   (27, "fp64", True, True), (34, "fp32", True, True)):
        A = R.laplace3d(N)
        spec = ras.partition("rcb", 1, grid=A.grid, seed=5, jitter=0.3)
        assert (A.n <= cap[storage]) == fits, (N, storage, A.n, cap)
        if not fits:
            with pytest.raises(ras.RasError) as e:
                ras.Plan(A, spec, 0, ras.local("chol_sparse", storage))
            assert e.value.status == -8 and "LDS" in str(e.value)
            continue
        plan = ras.Plan(A, spec, 0, ras.local("chol_sparse", storage))
        for pass_ in (0, 1):
            sch = plan.sparse_schedule(0, pass_)
            assert A.n + sch["slots"] <= cap[storage], (N, storage, sch["slots"])
            if full:
                assert sch["min_block"] == 0 and sch["slots"] == 0, (N, storage, sch["min_block"])


def test_sparse_schedule_arguments():
    """The schedule queries reject a pass other than 0 / 1, a subdomain out of
    range and a plan without sparse factors; the lane layout keeps every slot
    of the vector and the block slots below the 16-bit item columns' markers."""
    _lib_or_skip()
    A = R.laplace2d(24)
    plan = ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol_sparse", "fp32"))
    for bad in ((0, 2), (0, -1), (4, 0), (-1, 0)):
        with pytest.raises(ras.RasError) as e:
            plan.sparse_schedule(*bad)
        assert e.value.status == -1
        with pytest.raises(ras.RasError) as e:
            plan.sparse_lanes(*bad)
        assert e.value.status == -1
    band = ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 1, ras.local("chol", "fp32"))
    for call in (band.sparse_schedule, band.sparse_lanes):
        with pytest.raises(ras.RasError) as e:
            call(0, 0)
        assert e.value.status == -6
    _, ptr, _ = plan.sets()
    for p in range(4):
        n = int(ptr[p + 1] - ptr[p])
        for pass_ in (0, 1):
            sch = plan.sparse_schedule(p, pass_)
            lay = plan.sparse_lanes(p, pass_)
            assert n + sch["slots"] < 0xFFFE
            cols = lay["col"]
            assert np.all((cols < n + sch["slots"]) | (cols >= 0xFFFE))
            assert np.all(lay["wave"][:, 1] % 2 == 0)  # two rounds per column word on the device


def test_sparse_factor_of_disconnected_local_matrices():
    """Subdomains whose local matrix falls apart (a block-diagonal A: many small
    independent systems) are ordered component by component."""
    _lib_or_skip()
    blocks = [R.laplace2d(7).scipy() for _ in range(60)] + [sp.identity(500, format="csr") * 3.0]
    M = sp.block_diag(blocks, format="csr")
    M.sort_indices()
    M.indptr = M.indptr.astype(np.int64)
    M.indices = M.indices.astype(np.int32)
    plan = ras.Plan(M, ras.partition("regular_1d", 2), 1, ras.local("chol_sparse", "fp64"))
    _, ptr, idx = plan.sets()
    for p in range(2):
        om = idx[ptr[p]:ptr[p + 1]]
        perm, rp, col, val, diag = plan.sparse_factor(p)
        assert np.array_equal(np.sort(perm), np.arange(om.size))
        L = sp.csr_matrix((val, col, rp), shape=(om.size, om.size)) + sp.diags(diag)
        Ap = M[om][:, om][perm][:, perm]
        assert abs(L @ L.T - Ap).max() <= 1e-12 * abs(Ap).max()


# ----------------------------------------------------------------------------- stop rule (Sec. 3.3.2)
def test_async_stop_rule():
    """After an asynchronous launch the exact residual is verified; the library
    resumes, stops or reports a limit / divergence by this rule (host only)."""
    _lib_or_skip()
    nxt = ras.async_next_step
    # detector fired and verification passes / fails -> converged / resume
    assert nxt("detected", 9e-9, 1e-8, 100, 1000) == "converged"
    assert nxt("detected", 1.1e-8, 1e-8, 100, 1000) == "resume"
    # equality is not below the tolerance (strict criterion)
    assert nxt("detected", 1e-8, 1e-8, 100, 1000) == "resume"
    # limits: local-solve count, kernel time limit, time passed after the kernel, ordered mode
    assert nxt("exhausted", 1e-3, 1e-8, 1000, 1000) == "limit"
    assert nxt("detected", 1e-3, 1e-8, 999, 1000) == "resume"
    assert nxt("time", 1e-3, 1e-8, 10, 1000) == "limit"
    assert nxt("detected", 1e-3, 1e-8, 10, 1000, elapsed_seconds=5.0, max_seconds=4.0) == "limit"
    assert nxt("detected", 1e-3, 1e-8, 10, 1000, elapsed_seconds=5.0, max_seconds=0.0) == "resume"
    assert nxt("running", 1e-3, 1e-8, 3, 3, ordered=True) == "limit"
    assert nxt("running", 1e-3, 1e-8, 1, 3, ordered=True) == "limit"
    # a converged verification wins over a limit hit at the same time
    assert nxt("time", 1e-9, 1e-8, 1000, 1000) == "converged"
    # divergence wins over everything
    assert nxt("diverged", 1e-9, 1e-8, 1, 1000) == "diverged"
    assert nxt("detected", float("nan"), 1e-8, 1, 1000) == "diverged"
    assert nxt("detected", float("inf"), 1e-8, 1000, 1000) == "diverged"
    # tolerance 0 never converges
    assert nxt("exhausted", 0.0, 0.0, 5, 5) == "limit"
    assert ras.final_status("converged") == 0
    assert ras.final_status("limit") == 1
    assert ras.final_status("diverged") == -7
    assert ras.final_status("resume") == -6


# ----------------------------------------------------------------------------- Robin transmission (ORAS)
def test_oras_argument_errors():
    _lib_or_skip()
    A = R.laplace2d(16)
    for loc in (ras.local("cg", "fp64", 4, robin_q=0.5), ras.local("chol", "fp64", robin_q=0.0),
                ras.local("chol", "fp64", robin_q=1.5), ras.local("chol_sparse", "fp64", robin_q=-1.0)):
        with pytest.raises(ras.RasError) as e:
            ras.Plan(A, ras.partition("regular_1d", 2), 1, loc)
        assert e.value.status == -1


def test_oras_host_factor_is_cholesky_of_robin_local_matrix():
    """The library's host factor of an ORAS plan is the Cholesky factor of the oracle's
    Robin local matrix (A[omega, omega] with the diagonal lowered by (1 - q) e)."""
    _lib_or_skip()
    g = R.gaussian_random_field_2d(40, 6.0, 21)
    A = R.tpfa2d(np.exp(2 * g), 10.0)
    owner = opart.regular_grid(A.grid, (2, 2))
    plan = ras.Plan(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 3, ras.local("chol", "fp64", robin_q=0.4))
    for p, (_, om, _) in enumerate(oover.subdomain_sets(A, owner, 3)):
        band, w = plan.factor(p)
        Ap = olocal.robin_local_matrix(A, om, 0.4).toarray()
        Lref = np.linalg.cholesky(Ap)
        n = om.size
        L = np.zeros((n, n))
        for i in range(n):
            for o in range(w + 1):
                j = i - w + o
                if j >= 0:
                    L[i, j] = band[i, o]
        assert np.max(np.abs(L - Lref)) <= 1e-12 * np.abs(Lref).max()
    plan.close()
