"""Synthetic SPD test problems, all seeded, all FP64.

Matrix conventions (shared by every consumer):
  * CSR with int64 row pointers, int32 column indices sorted and unique per
    row, float64 values;
  * grid unknowns in natural order  g = i + nx*(j + ny*k)  (x fastest);
  * Dirichlet boundary nodes are eliminated, no h^2 scaling.

The 2-D Laplace problem follows the paper's experimental section (Sec. 4.1):
stencil {-1,-1,4,-1,-1} at offsets {-N,-1,0,1,N}, random right-hand side.
The other generators are the same construction in 3-D and its
variable-coefficient finite-volume (two-point flux) form.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """A square sparse matrix plus the grid it was generated on."""

    indptr: np.ndarray  # int64 [n+1]
    indices: np.ndarray  # int32 [nnz]
    data: np.ndarray  # float64 [nnz]
    grid: tuple  # (nx, ny, nz); nz == 1 for 2-D

    @property
    def n(self) -> int:
        return int(self.indptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.scipy() @ x

    def coords(self) -> np.ndarray:
        """Integer grid coordinates (n, 3) of each unknown."""
        nx, ny, nz = self.grid
        g = np.arange(self.n, dtype=np.int64)
        return np.stack([g % nx, (g // nx) % ny, g // (nx * ny)], axis=1).astype(np.int64)


def _from_coo(rows, cols, vals, n, grid) -> CSR:
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    return CSR(
        indptr=m.indptr.astype(np.int64),
        indices=m.indices.astype(np.int32),
        data=m.data.astype(np.float64),
        grid=tuple(int(v) for v in grid),
    )


def _stencil(nx: int, ny: int, nz: int, diag: float) -> CSR:
    n = nx * ny * nz
    g = np.arange(n, dtype=np.int64)
    i, j, k = g % nx, (g // nx) % ny, g // (nx * ny)
    rows = [g]
    cols = [g]
    vals = [np.full(n, diag)]
    for axis_pos, extent, stride in ((i, nx, 1), (j, ny, nx), (k, nz, nx * ny)):
        if extent == 1:
            continue
        lo = axis_pos > 0
        hi = axis_pos < extent - 1
        rows += [g[lo], g[hi]]
        cols += [g[lo] - stride, g[hi] + stride]
        vals += [np.full(int(lo.sum()), -1.0), np.full(int(hi.sum()), -1.0)]
    return _from_coo(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n, (nx, ny, nz))


def laplace2d(N: int, M: int | None = None) -> CSR:
    """2-D 5-point Laplacian on an N x M interior grid (stencil of Sec. 4.1)."""
    return _stencil(N, N if M is None else M, 1, 4.0)


def laplace3d(N: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """3-D 7-point Laplacian on an N x ny x nz interior grid (N^3 by default;
    diagonal 6, six -1's)."""
    return _stencil(N, N if ny is None else ny, N if nz is None else nz, 6.0)


def _tpfa(k: np.ndarray, aniso: tuple) -> CSR:
    """Two-point-flux finite volumes for -div(K grad u), K = k * diag(aniso), h = 1.

    Interior face transmissibility = aniso_axis * harmonic mean of the two cell
    values; a Dirichlet wall face contributes aniso_axis * 2 k_cell (half cell).
    """
    shape = k.shape  # (nz, ny, nx) or (ny, nx)
    if k.ndim == 2:
        k = k[None, :, :]
        aniso = (aniso[0], aniso[1], 1.0)
    nz, ny, nx = k.shape
    n = nx * ny * nz
    kf = k.reshape(-1)  # natural order: x fastest
    g = np.arange(n, dtype=np.int64)
    i, j, kk = g % nx, (g // nx) % ny, g // (nx * ny)
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for axis_pos, extent, stride, a in ((i, nx, 1, aniso[0]), (j, ny, nx, aniso[1]), (kk, nz, nx * ny, aniso[2])):
        if extent == 1:
            continue
        hi = axis_pos < extent - 1
        c0 = g[hi]
        c1 = c0 + stride
        t = a * 2.0 * kf[c0] * kf[c1] / (kf[c0] + kf[c1])
        rows += [c0, c1]
        cols += [c1, c0]
        vals += [-t, -t]
        np.add.at(diag, c0, t)
        np.add.at(diag, c1, t)
        lo_wall = axis_pos == 0
        hi_wall = axis_pos == extent - 1
        diag[lo_wall] += a * 2.0 * kf[lo_wall]
        diag[hi_wall] += a * 2.0 * kf[hi_wall]
    rows.append(g)
    cols.append(g)
    vals.append(diag)
    del shape
    return _from_coo(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), n, (nx, ny, nz))


def tpfa2d(k: np.ndarray, aniso_x: float = 1.0) -> CSR:
    """Variable-coefficient 2-D diffusion, k given per cell as an (ny, nx) array."""
    return _tpfa(np.asarray(k, dtype=np.float64), (aniso_x, 1.0))


def tpfa3d(k: np.ndarray) -> CSR:
    """Variable-coefficient 3-D diffusion, k given per cell as an (nz, ny, nx) array."""
    return _tpfa(np.asarray(k, dtype=np.float64), (1.0, 1.0, 1.0))


def gaussian_random_field_2d(N: int, corr_len: float, seed: int) -> np.ndarray:
    """Periodic unit-variance Gaussian random field with covariance exp(-r^2/(2 l^2)).

    White noise N(0,1) is filtered in Fourier space by the square root of the
    covariance's spectral density, exp(-2 pi^2 l^2 |f|^2), then normalised to
    sample mean 0 and standard deviation 1.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N))
    f = np.fft.fftfreq(N)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    filt = np.exp(-math.pi**2 * corr_len**2 * f2)  # sqrt of exp(-2 pi^2 l^2 f^2)
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    g -= g.mean()
    g /= g.std()
    return g


def uniform_rhs(n: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def manufactured_rhs(A: CSR, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """x* ~ U[-1, 1] (seeded) and b = A x*."""
    xs = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return A.matvec(xs), xs


def sine_mode_2d(N: int, a: int, c: int) -> tuple[np.ndarray, float]:
    """Discrete sine eigenmode v(i,j) = sin(a pi (i+1)/(N+1)) sin(c pi (j+1)/(N+1))
    of the 5-point Laplacian and its eigenvalue 4 - 2cos(a pi/(N+1)) - 2cos(c pi/(N+1))."""
    t = np.arange(1, N + 1) / (N + 1)
    v = np.outer(np.sin(c * math.pi * t), np.sin(a * math.pi * t)).reshape(-1)  # row j, column i
    lam = 4.0 - 2.0 * math.cos(a * math.pi / (N + 1)) - 2.0 * math.cos(c * math.pi / (N + 1))
    return v, lam


def sine_mode_3d(N: int, a: int, c: int, e: int) -> tuple[np.ndarray, float]:
    t = np.arange(1, N + 1) / (N + 1)
    sx, sy, sz = (np.sin(m * math.pi * t) for m in (a, c, e))
    v = (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).reshape(-1)
    lam = 6.0 - 2.0 * sum(math.cos(m * math.pi / (N + 1)) for m in (a, c, e))
    return v, lam


# ---------------------------------------------------------------------------
# The five benchmark workloads (sizes, partition, overlap, local solver, tol).
# ---------------------------------------------------------------------------
CONFIGS = {
    "poisson2d_64_strips4": dict(
        dims=2, N=64, partition=("regular_1d", 4), overlap=2, local=("chol", "fp64", 0), tol=1e-10, mode="sync",
        rhs=("manufactured", 0)),
    "poisson2d_512_strips64": dict(
        dims=2, N=512, partition=("regular_1d", 64), overlap=4, local=("chol", "fp64", 0), tol=1e-8,
        mode="async", rhs=("uniform", 1)),
    "poisson2d_1024_8x8": dict(
        dims=2, N=1024, partition=("regular_2d", (8, 8)), overlap=4, local=("cg", "fp64", 10), tol=1e-8,
        mode="async", rhs=("uniform", 1)),
    "laplace3d_128_rcb256": dict(
        dims=3, N=128, partition=("rcb", 256, 3, 0.4), overlap=1, local=("cg", "fp32", 8), tol=1e-8,
        mode="async", rhs=("uniform", 2)),
    "diffusion2d_2048_16x16": dict(
        dims=2, N=2048, partition=("regular_2d", (16, 16)), overlap=4, local=("chol", "fp64", 0), tol=1e-8,
        mode="async", rhs=("uniform", 5), field=dict(sigma=2.0, corr_len=32.0, seed=4, aniso_x=10.0)),
}


def config_problem(name: str, N: int | None = None):
    """Build (A, b, cfg) for a named workload; N overrides the grid side (for
    smaller instances of the same recipe)."""
    cfg = dict(CONFIGS[name])
    side = cfg["N"] if N is None else int(N)
    cfg["N"] = side
    if "field" in cfg:
        fld = cfg["field"]
        g = gaussian_random_field_2d(side, fld["corr_len"], fld["seed"])
        A = tpfa2d(np.exp(fld["sigma"] * g), fld["aniso_x"])
    elif cfg["dims"] == 2:
        A = laplace2d(side)
    else:
        A = laplace3d(side)
    kind, seed = cfg["rhs"]
    if kind == "manufactured":
        b, xs = manufactured_rhs(A, seed)
        cfg["x_star"] = xs
    else:
        b = uniform_rhs(A.n, seed)
    return A, b, cfg


def serving_stream(count: int = 2000, seed: int = 6, arrival_seed: int = 7, rate: float = 1.0,
                   min2d: int = 32, max2d: int = 512, min3d: int = 16, max3d: int = 96) -> Iterator[dict]:
    """Lazily yield the serving workload: half 2-D five-point, half 3-D seven-point
    finite-volume systems with i.i.d. log-normal (sigma 1) cell coefficients,
    log-uniform sides, 1..8 uniform[0,1] right-hand sides each, Poisson arrivals
    at `rate` systems per second."""
    rng = np.random.default_rng(seed)
    kinds = rng.permutation(np.array([2] * (count // 2) + [3] * (count - count // 2)))
    arr = np.random.default_rng(arrival_seed)
    t = 0.0
    for idx in range(count):
        dims = int(kinds[idx])
        if dims == 2:
            side = int(round(math.exp(rng.uniform(math.log(min2d), math.log(max2d)))))
        else:
            side = int(round(math.exp(rng.uniform(math.log(min3d), math.log(max3d)))))
        nrhs = int(rng.integers(1, 9))
        sys_seed = int(rng.integers(0, 2**31 - 1))
        t += float(arr.exponential(1.0 / rate))
        yield dict(index=idx, dims=dims, side=side, nrhs=nrhs, seed=sys_seed, arrival=t)


def serving_system(spec: dict):
    """Materialise one serving-stream system: (A, B[nrhs, n], partition parts, overlap)."""
    rng = np.random.default_rng(spec["seed"])
    side, dims = spec["side"], spec["dims"]
    if dims == 2:
        A = tpfa2d(np.exp(rng.standard_normal((side, side))))
        parts = (max(1, round(side / 64)),) * 2
    else:
        A = tpfa3d(np.exp(rng.standard_normal((side, side, side))))
        parts = (max(1, round(side / 16)),) * 3
    B = rng.uniform(0.0, 1.0, (spec["nrhs"], A.n))
    return A, B, parts
