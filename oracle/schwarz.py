"""Oracle Schwarz iterations.  Test infrastructure only.

Restricted additive Schwarz (Sec. 2.1, after Cai and Sarkis): every subdomain
solves its local problem on its overlapping set, the values computed on
overlap points are discarded and only the owned points are written back, so no
weighting is needed and writes never collide.  Reading (the paper writes it in
prose only), correction form with x^0 = 0:

    r^k      = b - A x^k
    hist[k]  = ||r^k||_2 / ||b||_2           (relative residual, Sec. 3.3.2)
    stop when hist[k] < tau                   (global criterion, Sec. 3.3.2)
    x^{k+1}  = x^k + sum_p  Rtilde_p^T S_p( R_p r^k )

where R_p restricts to Omega_p and Rtilde_p^T writes back owned points only.
The synchronous variant (Sec. 2.1, Sec. 3.4) applies all subdomain updates of
a sweep from the same x^k.  Alg. 1's loop -- local solve, exchange, update,
convergence check -- is one sweep here.

The asynchronous variant (Sec. 2.1, Sec. 3.4) has no sweep barrier: each
subdomain solves with whatever neighbour values it last received.  Two
deterministic stand-ins are provided: restricted multiplicative Schwarz (one
in-place x, subdomains visited in order -- the asynchronous iteration executed
by a single worker in a fixed order) and a seeded event simulator with bounded
staleness.  Convergence detection for the asynchronous variants follows
Sec. 2.2 / Sec. 3.3.2: the local criterion ||r_p||^2 < tau^2 ||b_p||^2 over the
overlapping set, a centralized detector that ends the iteration once every
subdomain reports local convergence, then a verification of the global
criterion after termination (resuming if it fails).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse.linalg as spla

from . import residual as ores
from .local import LocalSolver, local_matrix, robin_local_matrix
from .overlap import subdomain_sets


@dataclasses.dataclass
class Subdomain:
    owned: np.ndarray  # global ids, ascending
    omega: np.ndarray  # global ids, ascending, superset of owned
    ext: np.ndarray  # next layer out
    pos: np.ndarray  # positions of `owned` inside `omega`
    solver: LocalSolver


class RAS:
    """Setup of the Schwarz solver: subdomains, local matrices, local solvers."""

    def __init__(self, A, owner: np.ndarray, gamma: int, local: str = "chol", storage: str = "fp64",
                 cg_iters: int = 0, robin_q: float | None = None):
        """robin_q: optimized RAS with Robin transmission (oracle.local.robin_local_matrix);
        None: RAS with the Dirichlet local matrices."""
        self.A = A
        self.M = A.scipy()
        self.owner = np.asarray(owner, dtype=np.int32)
        self.gamma = gamma
        self.subs = []
        for own, om, ext in subdomain_sets(A, self.owner, gamma):
            Ap = local_matrix(A, om) if robin_q is None else robin_local_matrix(A, om, robin_q)
            self.subs.append(Subdomain(own, om, ext, np.searchsorted(om, own), LocalSolver(Ap, local, storage, cg_iters)))

    @property
    def P(self) -> int:
        return len(self.subs)

    def residual(self, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """b - A x, compensated (oracle.residual)."""
        return ores.residual(self.M, x, b)

    def local_residual(self, p: int, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """R_p (b - A x): the rows of A on Omega_p read x on Omega_p and its external layer."""
        return ores.residual(self.M, x, b, self.subs[p].omega)

    # -- synchronous RAS -------------------------------------------------------------
    def sync(self, b: np.ndarray, tol: float, max_sweeps: int, x0: np.ndarray | None = None, pool=None):
        """Returns (x, hist, sweeps): hist[k] = ||b - A x^k|| / ||b||, sweeps = updates applied.
        pool: optional concurrent.futures executor; the local solves of one sweep are
        independent (they all read r^k), so they may run concurrently; their
        corrections are still added in subdomain order, so the result is the same."""
        x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
        bn = np.linalg.norm(b)
        hist = []
        k = 0
        while True:
            r = self.residual(x, b) if pool is None else self._residual_on(pool, x, b)
            hist.append(np.linalg.norm(r) / bn)
            if hist[-1] < tol or k == max_sweeps:
                return x, np.array(hist), k
            x_next = x.copy()
            if pool is None:
                deltas = (s.solver(r[s.omega]) for s in self.subs)
            else:
                deltas = pool.map(lambda s: s.solver(r[s.omega]), self.subs)
            for s, delta in zip(self.subs, deltas):
                x_next[s.owned] += delta[s.pos]
            x = x_next
            k += 1

    def _residual_on(self, pool, x: np.ndarray, b: np.ndarray) -> np.ndarray:
        """The residual in row chunks on a thread pool (each row computed as in residual())."""
        chunks = np.array_split(np.arange(self.M.shape[0]), 4 * max(1, getattr(pool, "_max_workers", 1)))
        parts = pool.map(lambda rows: ores.residual(self.M, x, b, rows), chunks)
        return np.concatenate(list(parts))

    # -- restricted multiplicative Schwarz (ordered, in place) -------------------------
    def ordered(self, b: np.ndarray, passes: int, x0: np.ndarray | None = None):
        """`passes` full passes over p = 0..P-1, each local residual recomputed from the
        current x.  Returns (x, hist) with hist[k] the relative residual before pass k."""
        x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
        bn = np.linalg.norm(b)
        hist = []
        for _ in range(passes):
            hist.append(np.linalg.norm(self.residual(x, b)) / bn)
            for p, s in enumerate(self.subs):
                delta = s.solver(self.local_residual(p, x, b))
                x[s.owned] += delta[s.pos]
        hist.append(np.linalg.norm(self.residual(x, b)) / bn)
        return x, np.array(hist)

    # -- seeded asynchronous simulator --------------------------------------------------
    def neighbours(self) -> list[np.ndarray]:
        """Subdomains owning a point that subdomain p's local rows read (Omega_p and
        its external layer), excluding p."""
        out = []
        for p, s in enumerate(self.subs):
            cols = self.M[s.omega].indices
            q = np.unique(self.owner[cols])
            out.append(q[q != p])
        return out

    def async_sim(self, b: np.ndarray, tol: float, seed: int, staleness: int = 3, max_updates: int = 10**6,
                  x0: np.ndarray | None = None, paused: set | None = None, pause_until: int = 0,
                  detect: str = "central"):
        """Event-driven asynchronous RAS with bounded staleness.

        Each event picks a subdomain at random; it reads every other subdomain's
        owned values from one of that subdomain's last `staleness` published
        versions (chosen at random), computes its local residual, records the local
        criterion, solves and publishes its owned values.  Centralized detection:
        once every subdomain's latest local criterion holds, the iteration stops and
        the global criterion is verified on the current x; if it fails the iteration
        resumes.  Decentralized detection (Sec. 2.2, after Bahi et al.): a subdomain
        raises its global flag when it and all its neighbours report local
        convergence, or when a neighbour's flag is up (flooding), and then stops
        updating; once every flag is up the global criterion is verified, and on
        failure all flags are cleared and the iteration resumes.  Estimate
        detection (the library's option, not the paper's): once every subdomain
        has updated since the last reset and the sum of the owned residuals each
        computed at its latest update is below tol^2 ||b||^2, the global
        criterion is verified; on failure the update marks are cleared.  Subdomains in
        `paused` take no events before event `pause_until` (forced staleness).
        Returns (x, info dict)."""
        rng = np.random.default_rng(seed)
        x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
        bn2 = float(b @ b)
        P = self.P
        versions = [[x[s.owned].copy()] for s in self.subs]
        conv = np.zeros(P, dtype=bool)
        gflag = np.zeros(P, dtype=bool)
        own2 = np.full(P, np.inf)  # owned residual^2 of each subdomain's latest update
        nbrs = self.neighbours() if detect == "decentral" else None
        counts = np.zeros(P, dtype=np.int64)
        verifications = 0
        for ev in range(max_updates):
            p = int(rng.integers(P))
            if paused and p in paused and ev < pause_until:
                continue
            if gflag[p]:
                continue
            view = x.copy()
            for q, sq in enumerate(self.subs):
                if q == p:
                    continue
                hist_q = versions[q]
                pick = hist_q[-1 - int(rng.integers(min(staleness, len(hist_q))))]
                view[sq.owned] = pick
            s = self.subs[p]
            rp = ores.residual(self.M, view, b, s.omega)
            conv[p] = float(rp @ rp) < tol * tol * float(b[s.omega] @ b[s.omega])
            own2[p] = float(rp[s.pos] @ rp[s.pos])
            if detect == "estimate":
                conv[p] = True  # the mark: updated since the last reset
            delta = s.solver(rp)
            x[s.owned] += delta[s.pos]
            versions[p].append(x[s.owned].copy())
            if len(versions[p]) > staleness:
                versions[p].pop(0)
            counts[p] += 1
            if detect == "decentral":
                nb = nbrs[p]
                if (conv[p] and conv[nb].all()) or gflag[nb].any():
                    gflag[p] = True
                if not gflag.all():
                    continue
                verifications += 1
                r = self.residual(x, b)
                if float(r @ r) < tol * tol * bn2:
                    return x, dict(converged=True, events=ev + 1, local_solves=counts, verifications=verifications,
                                   relres=np.sqrt(float(r @ r) / bn2))
                gflag[:] = False
                conv[:] = False
                continue
            if conv.all() and (detect != "estimate" or own2.sum() < tol * tol * bn2):
                verifications += 1
                r = self.residual(x, b)
                if float(r @ r) < tol * tol * bn2:
                    return x, dict(converged=True, events=ev + 1, local_solves=counts, verifications=verifications,
                                   relres=np.sqrt(float(r @ r) / bn2))
                conv[:] = False
        r = self.residual(x, b)
        return x, dict(converged=False, events=max_updates, local_solves=counts, verifications=verifications,
                       relres=np.sqrt(float(r @ r) / bn2))


    def async_timed(self, b: np.ndarray, tol: float, durations, offsets=None, pace: float = 0.0,
                    max_rounds: int = 10**6):
        """Timed asynchronous schedule (a model of the one-GPU persistent kernel).

        Subdomain p runs updates back to back, each taking durations[p]; the first
        starts at offsets[p].  An update reads x on Omega_p and its external layer
        when it starts and publishes its owned values when it ends (Sec. 2.1: the
        local solve works on whatever values are there when it reads).  Paced
        reads: before starting, p waits until every neighbour has published at
        least as many updates as p, for at most pace * durations[p]; pace = 0 never
        waits.  Events at equal times publish before they read.  Stops when the
        exact relative residual drops below tol after a publish, or when every
        subdomain has published max_rounds updates.  Returns (x, info) with the
        local-solve counts and the stop time."""
        import heapq

        P = self.P
        dur = np.asarray(durations, dtype=np.float64)
        off = np.zeros(P) if offsets is None else np.asarray(offsets, dtype=np.float64)
        nbrs = self.neighbours()
        x = np.zeros_like(b)
        bn = np.linalg.norm(b)
        counts = np.zeros(P, dtype=np.int64)
        views = {}
        waiting = {}  # p -> deadline
        ev = [(off[p], 1, p) for p in range(P)]  # (time, 0 publish / 1 read / 2 wait deadline, p)
        heapq.heapify(ev)

        def behind(p):
            return any(counts[q] < counts[p] for q in nbrs[p])

        def start(p, t):
            views[p] = x.copy()
            heapq.heappush(ev, (t + dur[p], 0, p))

        while ev:
            t, kind, p = heapq.heappop(ev)
            if kind == 1:
                if counts[p] >= max_rounds:
                    continue
                if pace > 0 and behind(p):
                    waiting[p] = t + pace * dur[p]
                    heapq.heappush(ev, (waiting[p], 2, p))
                else:
                    start(p, t)
            elif kind == 2:
                if waiting.get(p) == t:
                    del waiting[p]
                    start(p, t)
            else:
                s = self.subs[p]
                view = views.pop(p)
                rp = ores.residual(self.M, view, b, s.omega)
                x[s.owned] = view[s.owned] + s.solver(rp)[s.pos]
                counts[p] += 1
                if np.linalg.norm(self.residual(x, b)) < tol * bn:
                    return x, dict(converged=True, local_solves=counts, time=t)
                for q in [q for q in waiting if not behind(q)]:
                    del waiting[q]
                    start(q, t)
                heapq.heappush(ev, (t, 1, p))
        return x, dict(converged=False, local_solves=counts, time=t)


def direct_solve(A, b: np.ndarray) -> np.ndarray:
    """FP64 direct reference solution: dense LU for n <= 4096, sparse LU otherwise."""
    if A.n <= 4096:
        return np.linalg.solve(A.scipy().toarray(), b)
    return spla.splu(A.scipy().tocsc()).solve(b)


def relative_residual(A, x: np.ndarray, b: np.ndarray) -> float:
    """||b - A x|| / ||b|| with the compensated residual (the verification of Sec. 3.3.2)."""
    return ores.relative_residual(A.scipy(), x, b)
