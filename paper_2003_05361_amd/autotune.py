"""Choice of the exact local solver by measurement.

Banded and sparse Cholesky factors of a local matrix give the same local solution
up to rounding (Sec. 3.3.1: the local problems are solved exactly), so the RAS
iteration and its sweep count to a tolerance are the same with either; only the
time per sweep differs.  Which one is faster depends on the subdomains: the
band streams n (w + 1) entries per triangular pass through LDS stages, while
the sparse factor (nested dissection) holds fewer entries but keeps the local
vector resident in LDS, which bounds the subdomain size.  `exact_local` times a
few synchronous sweeps of every feasible candidate on the caller's system and
returns the faster one; choices are cached per problem shape for the process.
The storage (precision) of the factor stays the caller's choice.
"""
from __future__ import annotations

import paper_2003_05361_amd as ras

_cache: dict = {}


def _key(A, part: dict, overlap: int, storage: str) -> tuple:
    spec = tuple(sorted((k, str(v)) for k, v in part.items() if k != "owner"))
    return (int(A.n), int(A.indptr[-1]), spec, int(overlap), storage)


def exact_local(A, part: dict, overlap: int, b, storage: str = "fp64", sweeps: int = 20, stream=None,
                use_cache: bool = True) -> tuple[dict, dict]:
    """Returns (local solver spec for ras.setup, report).  b: the right-hand side
    on the device (the timed sweeps start from x = 0).  The report lists every
    candidate's milliseconds per synchronous sweep (None where the candidate
    does not apply: the sparse solver keeps at most ras.sparse_max_rows(storage)
    local rows and has no FP16 storage)."""
    key = _key(A, part, overlap, storage)
    if use_cache and key in _cache:
        kind, report = _cache[key]
        return ras.local(kind, storage), dict(report, cached=True)
    times = {}
    for kind in ("chol", "chol_sparse"):
        try:
            h = ras.setup(A, part, overlap, ras.local(kind, storage), stream=stream)
        except ras.RasError:
            times[kind] = None
            continue
        try:
            h.solve(b, tol=0.0, mode="sync", max_sweeps=2)  # warm-up
            _, info = h.solve(b, tol=0.0, mode="sync", max_sweeps=int(sweeps))
            i = info[0]
            # the synchronous kernel computes one speculative update after its last sweep
            times[kind] = 1e3 * i["kernel_seconds"] / (i["sweeps"] + 1)
        finally:
            h.close()
    feasible = {k: v for k, v in times.items() if v is not None}
    if not feasible:
        raise ras.RasError(-1, "no exact local solver applies to this problem")
    kind = min(feasible, key=feasible.get)
    report = {"ms_per_sweep": times, "choice": kind, "sweeps": int(sweeps), "cached": False}
    _cache[key] = (kind, report)
    return ras.local(kind, storage), report
