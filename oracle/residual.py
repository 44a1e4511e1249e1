"""Oracle outer residual b - A x.  Test infrastructure only.

Sec. 3.3.2 measures convergence by the relative residual ||b - A x|| / ||b||
and does not say in which precision it is evaluated.  Reading: every row of
the outer residual is accumulated in compensated (double-word) arithmetic --
the Dot2 algorithm of Ogita, Rump and Oishi ("Accurate sum and dot product",
SIAM J. Sci. Comput. 26, 2005) -- so that the result is as accurate as if it
had been computed in twice float64's precision and then rounded.  Near
convergence b - A x cancels; a plain float64 sum then carries an absolute error
of about eps * (|A| |x|)_i per row, which on strongly varying coefficients is as
large as the tolerance itself.

Steps (per row, terms in stored column order): s = b_i, c = 0; for each stored
a_ij: (p, e) = TwoProduct(a_ij, x_j), (s, t) = TwoSum(s, -p), c = c + (t - e);
result s + c.  TwoProduct is Dekker's (1971) with Veltkamp's splitting (numpy
has no fused multiply-add); TwoSum is Knuth's.  Both are exact for finite
values away from overflow.
"""
from __future__ import annotations

import numpy as np

_SPLITTER = 134217729.0  # 2^27 + 1: Veltkamp's splitting of a float64 into two 26-bit halves


def two_sum(a: np.ndarray, b: np.ndarray):
    """s + t == a + b exactly, s = fl(a + b) (Knuth)."""
    s = a + b
    z = s - a
    t = (a - (s - z)) + (b - z)
    return s, t


def _split(a: np.ndarray):
    c = _SPLITTER * a
    hi = c - (c - a)
    return hi, a - hi


def two_product(a: np.ndarray, b: np.ndarray):
    """p + e == a * b exactly, p = fl(a * b) (Dekker, Veltkamp splitting)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = al * bl - (((p - ah * bh) - al * bh) - ah * bl)
    return p, e


def residual(M, x: np.ndarray, b: np.ndarray, rows: np.ndarray | None = None) -> np.ndarray:
    """Compensated b - M x for all rows of the CSR matrix M, or for the listed
    rows only (b and x are full-length vectors either way)."""
    indptr = np.asarray(M.indptr, dtype=np.int64)
    indices = np.asarray(M.indices)
    data = np.asarray(M.data, dtype=np.float64)
    r_ids = np.arange(M.shape[0]) if rows is None else np.asarray(rows, dtype=np.int64)
    start = indptr[r_ids]
    length = indptr[r_ids + 1] - start
    s = np.array(b[r_ids], dtype=np.float64)
    c = np.zeros_like(s)
    for k in range(int(length.max(initial=0))):
        live = np.flatnonzero(length > k)
        e_ids = start[live] + k
        p, pe = two_product(data[e_ids], x[indices[e_ids]])
        s_new, t = two_sum(s[live], -p)
        s[live] = s_new
        c[live] += t - pe
    return s + c


def relative_residual(M, x: np.ndarray, b: np.ndarray) -> float:
    r = residual(M, x, b)
    return float(np.linalg.norm(r) / np.linalg.norm(b))
