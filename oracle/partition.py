"""Oracle partitioners: point -> owning subdomain (int32).  Test infrastructure only.

Sec. 3.2.1 of the paper describes regular 1-D strips (at most two neighbours;
information needs N-1 iterations to cross N strips), regular 2-D boxes (at most
four neighbours) and an edge-cut-minimising graph partitioner.  The graph
partitioner is third-party software that is not reproduced; recursive
coordinate bisection with seeded, jittered part weights stands in for it.

Readings (the paper gives no formulas for any of these):
  * regular-1d(P): part p owns rows [floor(p n/P), floor((p+1) n/P)) of the
    natural ordering -- grid-row strips when P divides the row count;
  * regular grid (px, py[, pz]): axis bounds b_i = floor(i N_axis / p_axis),
    subdomain id p = ix + px (iy + py iz), x fastest;
  * RCB: part weights w_q = 1 + jitter (2 u_q - 1) with u_q the q-th SplitMix64
    output (Steele, Lea, Flood, OOPSLA 2014) shifted right by 11 and scaled by
    2^-53; split the largest-extent axis (ties: lowest axis), order points by
    (coordinate, global id), cut = floor(|S| W_left / W + 0.5) clamped so that
    every part keeps at least one point.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64_outputs(seed: int, count: int) -> list[int]:
    """The first `count` outputs of SplitMix64 started from state `seed`."""
    state = seed & MASK64
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def rcb_weights(P: int, seed: int, jitter: float) -> list[float]:
    """Jittered target weights of the P parts."""
    ws = []
    for z in splitmix64_outputs(seed, P):
        u = float(z >> 11) * (2.0 ** -53)
        ws.append(1.0 + jitter * (2.0 * u - 1.0))
    return ws


def regular_1d(n: int, P: int) -> np.ndarray:
    owner = np.empty(n, dtype=np.int32)
    for p in range(P):
        lo = (p * n) // P
        hi = ((p + 1) * n) // P
        owner[lo:hi] = p
    return owner


def _axis_part(extent: int, parts: int) -> np.ndarray:
    """Index of the axis slab each coordinate falls in."""
    slab = np.empty(extent, dtype=np.int64)
    for s in range(parts):
        lo = (s * extent) // parts
        hi = ((s + 1) * extent) // parts
        slab[lo:hi] = s
    return slab


def regular_grid(grid: tuple, parts: tuple) -> np.ndarray:
    """Regular 2-D / 3-D box partition of an nx x ny x nz natural-order grid."""
    nx, ny, nz = (tuple(grid) + (1, 1))[:3]
    px, py, pz = (tuple(parts) + (1, 1))[:3]
    sx, sy, sz = _axis_part(nx, px), _axis_part(ny, py), _axis_part(nz, pz)
    owner = np.empty(nx * ny * nz, dtype=np.int32)
    for k in range(nz):
        for j in range(ny):
            base = nx * (j + ny * k)
            owner[base:base + nx] = sx + px * (sy[j] + py * sz[k])
    return owner


def rcb(coords: np.ndarray, P: int, seed: int, jitter: float) -> np.ndarray:
    """Recursive coordinate bisection of integer points `coords` (n, d) into P parts."""
    n = coords.shape[0]
    if not 1 <= P <= n:
        raise ValueError("RCB needs 1 <= P <= n")
    w = rcb_weights(P, seed, jitter)
    owner = np.full(n, -1, dtype=np.int32)
    stack = [(np.arange(n, dtype=np.int64), 0, P)]
    while stack:
        S, p0, m = stack.pop()
        if m == 1:
            owner[S] = p0
            continue
        ml = m // 2
        ext = [int(coords[S, a].max() - coords[S, a].min()) for a in range(coords.shape[1])]
        axis = int(np.argmax(ext))  # first maximum = lowest axis on ties
        order = np.lexsort((S, coords[S, axis]))  # primary key: coordinate, then id
        S = S[order]
        Wl = 0.0
        for q in range(p0, p0 + ml):
            Wl += w[q]
        W = Wl
        for q in range(p0 + ml, p0 + m):
            W += w[q]
        cut = int(np.floor(len(S) * Wl / W + 0.5))
        cut = min(max(cut, ml), len(S) - (m - ml))
        stack.append((S[:cut], p0, ml))
        stack.append((S[cut:], p0 + ml, m - ml))
    return owner


def make_owner(A, kind: str, arg) -> np.ndarray:
    """Dispatch on the partition description used by the workloads."""
    if kind == "regular_1d":
        return regular_1d(A.n, int(arg))
    if kind in ("regular_2d", "regular_3d"):
        return regular_grid(A.grid, tuple(arg))
    if kind == "rcb":
        P, seed, jitter = arg
        return rcb(A.coords(), int(P), int(seed), float(jitter))
    if kind == "explicit":
        return np.asarray(arg, dtype=np.int32)
    raise ValueError(kind)
