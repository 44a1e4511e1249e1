"""ras_solve_noalloc (the solve whose workspace is the library's fixed device
scratch, for callers that cannot allocate) against ras_solve, through the C ABI:
the same kernels on the same inputs give the same iterates, also on a second
call with a smaller system (the scratch keeps the first call's contents), and a
workspace larger than the scratch is refused before any device work."""
import sys

import numpy as np
import pytest

import ras_inputs as R
from oracle import schwarz

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cuda(v):
    import torch

    return torch.tensor(np.ascontiguousarray(v), dtype=torch.float64, device="cuda")


def _ras():
    import paper_2003_05361_amd as ras

    ras.lib()
    return ras


@pytest.mark.parametrize("loc,storage,k", [("cg", "fp64", 6), ("chol", "fp32", 0), ("chol_sparse", "fp64", 0)])
def test_noalloc_equals_solve_twice_second_smaller(loc, storage, k):
    import torch

    ras = _ras()
    cases = [(R.laplace2d(96), (4, 4), 3, 51), (R.laplace2d(40, 36), (2, 3), 2, 52)]  # second call smaller
    for A, parts, gamma, seed in cases:
        _say(f"case: noalloc {loc} {storage} n={A.n}")
        b = R.uniform_rhs(A.n, seed)
        h = ras.setup(A, ras.partition("regular_2d", parts, grid=A.grid), gamma, ras.local(loc, storage, k))
        bt = _cuda(b)
        x_ref, i_ref = h.solve(bt, tol=1e-9, mode="sync", max_sweeps=20000)
        x_na, i_na = h.solve(bt, tol=1e-9, mode="sync", max_sweeps=20000, noalloc=True)
        assert i_na[0]["converged"] and i_na[0]["sweeps"] == i_ref[0]["sweeps"]
        assert torch.equal(x_na, x_ref)
        _, h_ref = h.residual_history()
        # asynchronous through the fixed scratch: converges and verifies
        xa, ia = h.solve(bt, tol=1e-9, mode="async", max_sweeps=200000, max_seconds=60, noalloc=True)
        assert ia[0]["converged"]
        assert schwarz.relative_residual(A, xa.cpu().numpy(), b) < 1e-9
        h.close()


def test_noalloc_multi_rhs_equals_solve():
    import torch

    ras = _ras()
    _say("case: noalloc multi rhs")
    A = R.laplace2d(50)
    B = np.stack([R.uniform_rhs(A.n, s) for s in (61, 62, 63)])
    h = ras.setup(A, ras.partition("regular_2d", (3, 3), grid=A.grid), 2, ras.local("cg", "fp64", 5))
    X1, _ = h.solve(_cuda(B), tol=1e-8, mode="sync", max_sweeps=100000)
    X2, _ = h.solve(_cuda(B), tol=1e-8, mode="sync", max_sweeps=100000, noalloc=True)
    assert torch.equal(X1, X2)
    h.close()


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    ras = _ras()
    _say("case: noalloc too large")
    A = R.laplace2d(1500)  # sync: second iterate 18 MB + local vectors > 20 MB: beyond the 32 MiB scratch
    b = _cuda(R.uniform_rhs(A.n, 64))
    h = ras.setup(A, ras.partition("regular_2d", (8, 8), grid=A.grid), 2, ras.local("cg", "fp64", 2))
    with pytest.raises(ras.RasError) as e:
        h.solve(b, tol=1e-8, mode="sync", max_sweeps=10, noalloc=True)
    assert e.value.status == -4 and "no-allocation scratch" in str(e.value)
    # the ordinary entry point still solves it
    _, info = h.solve(b, tol=0.0, mode="sync", max_sweeps=2)
    assert info[0]["sweeps"] == 2
    h.close()
