"""Oracle overlap construction.  Test infrastructure only.

Sec. 2.1 (Fig. 1) defines overlap gamma: a subdomain's local problem includes,
besides its own (owned) points, the points reached by gamma layers around them;
the next layer out ("external interface" points) is where the exchanged
information comes from.  Reading: layers are breadth-first layers over the
stored off-diagonal pattern of A (graph distance), local order is ascending
global id.
"""
from __future__ import annotations

import numpy as np


def _neighbours(indptr: np.ndarray, indices: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """All column indices stored in the given rows (with repeats)."""
    if rows.size == 0:
        return rows
    starts = indptr[rows]
    counts = indptr[rows + 1] - starts
    offs = np.repeat(starts - np.concatenate(([0], np.cumsum(counts)[:-1])), counts)
    return indices[np.arange(counts.sum()) + offs]


def bfs_layers(A, seeds: np.ndarray, layers: int) -> list[np.ndarray]:
    """Breadth-first layers: result[0] = seeds, result[l] = points at graph distance l."""
    visited = np.zeros(A.n, dtype=bool)
    visited[seeds] = True
    frontier = np.asarray(seeds, dtype=np.int64)
    out = [np.sort(frontier)]
    for _ in range(layers):
        nb = np.unique(_neighbours(A.indptr, A.indices, frontier))
        new = nb[~visited[nb]]
        visited[new] = True
        out.append(new.astype(np.int64))
        frontier = new
    return out


def subdomain_sets(A, owner: np.ndarray, gamma: int):
    """Per subdomain p: (owned O_p, overlapping Omega_p, external ext(Omega_p)),
    each an ascending int64 array of global ids."""
    P = int(owner.max()) + 1
    res = []
    for p in range(P):
        own = np.flatnonzero(owner == p)
        lay = bfs_layers(A, own, gamma + 1)
        omega = np.sort(np.concatenate(lay[: gamma + 1]))
        ext = np.sort(lay[gamma + 1])
        res.append((own, omega, ext))
    return res


def flatten_sets(sets) -> tuple[np.ndarray, np.ndarray]:
    """omega_ptr (int64, P+1) and omega_idx (int32) in the layout the library exports."""
    ptr = np.zeros(len(sets) + 1, dtype=np.int64)
    for p, (_, om, _) in enumerate(sets):
        ptr[p + 1] = ptr[p] + om.size
    idx = np.concatenate([om for (_, om, _) in sets]).astype(np.int32)
    return ptr, idx


def comm_volume(owner: np.ndarray, sets) -> np.ndarray:
    """Sec. 3.2.1 (Fig. 2): P x P communication volume.  Entry [p, q], q != p,
    counts the points of Omega_p and of its external layer that subdomain q
    owns, i.e. the values p needs from q to form its local problem once; the
    diagonal is 0.  Rows are receivers, columns senders."""
    P = len(sets)
    vol = np.zeros((P, P), dtype=np.int64)
    for p, (_, omega, ext) in enumerate(sets):
        for i in list(omega) + list(ext):
            q = int(owner[i])
            if q != p:
                vol[p, q] += 1
    return vol
