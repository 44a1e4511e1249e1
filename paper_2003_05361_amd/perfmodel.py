"""Algorithmic HBM-byte model of one local solve (streaming model: each array
touched the minimum number of times per step, no reuse across CG iterations).

The three parts follow the update of Sec. 2.1 (Eq. 3, restricted form):
restriction of the residual onto Omega_p, the local solve, and the restricted
prolongation onto the owned points.
"""
from __future__ import annotations

import numpy as np

_SOLVE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}


def subdomain_shapes(plan, indptr, sparse: bool = False) -> list:
    """[n_p, owned_p, K_p, w_p] per subdomain of a host plan: local rows, owned
    rows, widest stored row of A over Omega_p and the local half-bandwidth;
    with sparse=True (a sparse Cholesky plan) also nnz of the strictly lower
    part of the factor."""
    owner, ptr, idx = plan.sets()
    shapes = []
    for p in range(len(ptr) - 1):
        om = idx[ptr[p]:ptr[p + 1]]
        n_own = int(np.count_nonzero(owner[om] == p))
        K = int(np.max(indptr[om + 1] - indptr[om])) if om.size else 0
        sh = [int(om.size), n_own, K, plan.band_width(p)]
        if sparse:
            sh.append(int(plan.sparse_factor(p)[1][-1]))
        shapes.append(sh)
    return shapes


def local_solve_parts(shape, kind: str, storage: str, k: int) -> tuple[float, float, float]:
    """(residual, local solve, prolongation) bytes of one local solve.

    residual: K (value, column) pairs and the K read values of x per local row,
    plus b and the local right-hand side; local solve: k CG iterations over the
    ELL rows and five vectors, or the band factor streamed forward and backward
    plus right-hand side and solution (sparse: the factor entries with their
    columns and row records, per pass); prolongation: read x and the correction,
    write x, per owned row."""
    n, n_own, K, w = shape[:4]
    s = 8 if storage == "fp64" else 4
    res = n * (12 * K + 16)
    pro = n_own * (16 + s)
    if kind == "cg":
        loc = k * n * (K * (s + 4) + 11 * s)
    elif kind == "chol_sparse":
        # per pass: every stored entry (the scaled diagonal included) as value + column,
        # one 16-byte row record; the local vector read before and written after
        sl = _SOLVE_BYTES[storage]
        loc = 2 * ((shape[4] + n) * (sl + 4) + 16 * n) + 2 * n * s
    else:
        sl = _SOLVE_BYTES[storage]
        loc = 2 * n * (w + 1) * sl + 4 * n * s + (2 * n * 4 if storage == "fp16" else 0)
    return float(res), float(loc), float(pro)


def bytes_per_local_solve(shapes, kind: str, storage: str, k: int) -> list:
    return [sum(local_solve_parts(sh, kind, storage, k)) for sh in shapes]
