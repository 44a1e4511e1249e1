"""Oracle local subdomain problems and local solvers.  Test infrastructure only.

Sec. 3.2.2: each subdomain holds the local matrix on its overlapping set.
Reading: A_p = A[Omega_p, Omega_p], a principal submatrix (homogeneous
Dirichlet on the artificial boundary), rows and columns in ascending global id.

Sec. 3.3.1: the local problem is solved either directly -- a Cholesky
factorisation computed once, then triangular solves in every iteration -- or
iteratively (CG among others).  Readings:
  * direct: the factor is the banded Cholesky factor of A_p, lower half-width
    w = max_i (i - min{j : (A_p)_ij stored}); scipy's LAPACK band routines do
    the factor and the two triangular solves;
  * iterative: k steps of Hestenes-Stiefel CG from a zero initial guess, no
    inner tolerance, stopped early only on breakdown (rho == 0 or p'Ap <= 0);
  * FP32 storage: factor (or matrix) values rounded to float32, all local
    arithmetic in float32, the correction returned in FP64;
  * FP16 with per-row scaling: s_i = float32(max_j |L_ij|), stored entries
    fp16_RNE(L_ij / s_i) computed from FP64, dequantised to float32 as
    float32(Lhat_ij) * s_i, triangular solves in float32.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack
import scipy.sparse as sp


def local_matrix(A, omega: np.ndarray) -> sp.csr_matrix:
    M = A.scipy()[omega][:, omega].tocsr()
    M.sort_indices()
    return M


def outside_coupling(A, omega: np.ndarray) -> np.ndarray:
    """e_i = sum of |a_ij| over the columns j of row omega[i] that lie outside omega."""
    M = A.scipy()
    inside = np.zeros(A.n, dtype=bool)
    inside[omega] = True
    rows = abs(M[omega]).tocsr()
    e = np.zeros(omega.size)
    for i in range(omega.size):
        cols = rows.indices[rows.indptr[i]:rows.indptr[i + 1]]
        vals = rows.data[rows.indptr[i]:rows.indptr[i + 1]]
        e[i] = vals[~inside[cols]].sum()
    return e


def robin_local_matrix(A, omega: np.ndarray, q: float) -> sp.csr_matrix:
    """Optimized Schwarz (Sec. 5 names it as future work) with a Robin condition on the
    artificial boundary, in algebraic form.  Reading: A[omega, omega] with the
    diagonal lowered by (1 - q) e_i, e_i the row's coupling to points outside omega
    (q = 1: the Dirichlet local matrix of RAS; smaller q moves the condition from
    Dirichlet towards Neumann)."""
    Ap = local_matrix(A, omega)
    return (Ap - sp.diags((1.0 - q) * outside_coupling(A, omega))).tocsr()


def lower_bandwidth(Ap: sp.csr_matrix) -> int:
    """w = max over stored entries (i, j) of i - j."""
    rows = np.repeat(np.arange(Ap.shape[0]), np.diff(Ap.indptr))
    return int(max(0, (rows - Ap.indices).max(initial=0)))


def band_lower_form(Ap: sp.csr_matrix, w: int) -> np.ndarray:
    """LAPACK lower band storage: ab[k, i] = A_p[i + k, i]."""
    n = Ap.shape[0]
    ab = np.zeros((w + 1, n))
    C = Ap.tocoo()
    m = (C.row >= C.col) & (C.row - C.col <= w)
    ab[C.row[m] - C.col[m], C.col[m]] = C.data[m]
    return ab


def band_cholesky(Ap: sp.csr_matrix):
    """Lower banded Cholesky factor of A_p: (cb, w) with cb in LAPACK lower band form."""
    w = lower_bandwidth(Ap)
    cb = sla.cholesky_banded(band_lower_form(Ap, w), lower=True)
    return cb, w


def band_to_dense_lower(cb: np.ndarray) -> np.ndarray:
    w1, n = cb.shape
    L = np.zeros((n, n), dtype=cb.dtype)
    for k in range(w1):
        idx = np.arange(n - k)
        L[idx + k, idx] = cb[k, : n - k]
    return L


def chol_solve_fp64(cb: np.ndarray, r: np.ndarray) -> np.ndarray:
    return sla.cho_solve_banded((cb, True), r)


def band_row_index(cb: np.ndarray) -> np.ndarray:
    """Row index i = j + k of every band slot cb[k, j] (slots past the end map to n)."""
    w1, n = cb.shape
    return np.minimum(np.arange(n)[None, :] + np.arange(w1)[:, None], n)


def quantize_rows_fp16(cb: np.ndarray):
    """Per-row scaled FP16 copy of a lower band factor: (Lhat float16 band, s float32[n])."""
    w1, n = cb.shape
    rows = band_row_index(cb)
    rmax = np.zeros(n + 1)
    np.maximum.at(rmax, rows.reshape(-1), np.abs(cb).reshape(-1))
    s = rmax[:n].astype(np.float32)
    s = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    s_ext = np.concatenate([s.astype(np.float64), [1.0]])
    Lhat = (cb / s_ext[rows]).astype(np.float16)
    return Lhat, s


def dequantize_rows_fp16(Lhat: np.ndarray, s: np.ndarray) -> np.ndarray:
    rows = band_row_index(Lhat)
    s_ext = np.concatenate([s, [np.float32(1.0)]]).astype(np.float32)
    out = Lhat.astype(np.float32) * s_ext[rows]
    assert out.dtype == np.float32
    return out


def chol_solve_lowp(cb32: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Forward (L y = r) then backward (L^T x = y) banded triangular solves in float32."""
    assert cb32.dtype == np.float32
    y, info = lapack.stbtrs(cb32, r.astype(np.float32)[:, None], uplo="L", trans="N", diag="N")
    assert info == 0
    x, info = lapack.stbtrs(cb32, y, uplo="L", trans="T", diag="N")
    assert info == 0 and x.dtype == np.float32
    return x[:, 0].astype(np.float64)


def cg_fixed(Ap, r: np.ndarray, k: int, dtype=np.float64) -> np.ndarray:
    """k steps of Hestenes-Stiefel CG on A_p delta = r from delta = 0."""
    M = Ap.astype(dtype)
    res = r.astype(dtype)
    delta = np.zeros_like(res)
    p = res.copy()
    rho = res @ res
    for _ in range(k):
        q = M @ p
        sigma = p @ q
        if rho == 0 or sigma <= 0:
            break
        alpha = rho / sigma
        delta = delta + alpha * p
        res = res - alpha * q
        rho_new = res @ res
        p = res + (rho_new / rho) * p
        rho = rho_new
    return delta.astype(np.float64)


class LocalSolver:
    """S_p: the local solve of one subdomain, configured once (setup) and applied
    to a restricted residual every iteration."""

    def __init__(self, Ap: sp.csr_matrix, kind: str, storage: str = "fp64", cg_iters: int = 0):
        self.kind, self.storage, self.k = kind, storage, cg_iters
        self.Ap = Ap
        if kind == "chol":
            cb, w = band_cholesky(Ap)
            self.cb, self.w = cb, w
            if storage == "fp32":
                self.cb32 = cb.astype(np.float32)
            elif storage == "fp16":
                self.Lhat, self.scale = quantize_rows_fp16(cb)
                self.cb32 = dequantize_rows_fp16(self.Lhat, self.scale)
            elif storage != "fp64":
                raise ValueError(storage)
        elif kind != "cg":
            raise ValueError(kind)

    def __call__(self, r: np.ndarray) -> np.ndarray:
        if self.kind == "chol":
            if self.storage == "fp64":
                return chol_solve_fp64(self.cb, r)
            return chol_solve_lowp(self.cb32, r)
        return cg_fixed(self.Ap, r, self.k, np.float64 if self.storage == "fp64" else np.float32)
