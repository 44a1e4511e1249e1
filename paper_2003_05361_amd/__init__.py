"""Python binding of the MI355X restricted additive Schwarz library (libras.so).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels and C++ setup code.  torch supplies device memory and streams.  The
library must have been built (``python -m paper_2003_05361_amd.build``); a
missing library is an error, never a fallback.

    import paper_2003_05361_amd as ras
    h = ras.setup(A, ras.partition("regular_2d", (8, 8), grid=A.grid), overlap=4,
                  local=ras.local("cg", "fp64", 10))
    x, info = h.solve(b_cuda, tol=1e-8, mode="async")
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RAS_LIBRARY may name another build of the same library (the host-sanitizer
# build of paper_2003_05361_amd.hostsan); by default the in-tree libras.so
LIB_PATH = os.environ.get("RAS_LIBRARY") or os.path.join(_HERE, "_lib", "libras.so")

# ----------------------------------------------------------------------------- C mirrors
RAS_OK, RAS_NOT_CONVERGED, RAS_PENDING = 0, 1, 2
# why a persistent launch stopped a right-hand side, and the host's next step (Sec. 3.3.2)
KSTOP = {"running": 0, "detected": 1, "time": 2, "exhausted": 3, "diverged": 4}
STEPS = {0: "converged", 1: "resume", 2: "diverged", 3: "limit"}
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "E_ARG", -2: "E_PATTERN", -3: "E_NOT_SPD",
                -4: "E_NOMEM", -5: "E_HIP", -6: "E_STATE", -7: "E_DIVERGED", -8: "E_UNSUPPORTED"}
PART_KINDS = {"regular_1d": 0, "regular_2d": 1, "regular_3d": 2, "rcb": 3, "explicit": 4}
LOCAL_KINDS = {"chol": 0, "cg": 1, "chol_sparse": 2}
STORAGES = {"fp64": 0, "fp32": 1, "fp16": 2}
MODES = {"sync": 0, "async": 1, "ordered": 2}
DETECT = {"central": 0, "decentral": 1, "estimate": 2}
# size of the library's fixed device workspace of ras_solve_noalloc (per device)
NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024
# asynchronous mode: neighbour wait budget before a read, in units of the previous update's time
# (0 = free running, negative = the library's choice per local solver)
DEFAULT_PACE = -1.0


class CSRStruct(C.Structure):
    _fields_ = [("n", C.c_int64), ("row_ptr", C.POINTER(C.c_int64)), ("col", C.POINTER(C.c_int32)),
                ("val", C.POINTER(C.c_double))]


class PartitionStruct(C.Structure):
    _fields_ = [("kind", C.c_int32), ("grid", C.c_int32 * 3), ("parts", C.c_int32 * 3), ("reserved", C.c_int32),
                ("seed", C.c_uint64), ("jitter", C.c_double), ("owner", C.POINTER(C.c_int32))]


class LocalStruct(C.Structure):
    _fields_ = [("kind", C.c_int32), ("cg_iters", C.c_int32), ("storage", C.c_int32), ("transmission", C.c_int32),
                ("robin_q", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("detect", C.c_int32), ("tol", C.c_double), ("max_sweeps", C.c_int64),
                ("max_seconds", C.c_double), ("workgroups", C.c_int32), ("team", C.c_int32), ("pace", C.c_double),
                ("detect_factor", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("converged", C.c_int32), ("launches", C.c_int32), ("sweeps", C.c_int64),
                ("total_local_solves", C.c_int64), ("min_local_solves", C.c_int64),
                ("max_local_solves", C.c_int64), ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("kernel_seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("parts", C.c_int32), ("max_ell_width", C.c_int32),
                ("sum_local_rows", C.c_int64), ("min_local_rows", C.c_int64), ("max_local_rows", C.c_int64),
                ("max_band", C.c_int32), ("reserved", C.c_int32), ("band_entries", C.c_int64),
                ("device_bytes", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# every symbol the header declares, with its ctypes signature
_P = C.c_void_p
SIGNATURES = {
    "ras_plan_create": (C.c_int, [C.POINTER(CSRStruct), C.POINTER(PartitionStruct), C.c_int32,
                                  C.POINTER(LocalStruct), C.POINTER(_P)]),
    "ras_plan_get_stats": (C.c_int, [_P, C.POINTER(PlanStats)]),
    "ras_plan_sets": (C.c_int, [_P, _P, _P, _P]),
    "ras_plan_comm_volume": (C.c_int, [_P, _P]),
    "ras_plan_factor": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "ras_plan_factor_fp16": (C.c_int, [_P, C.c_int32, _P, _P]),
    "ras_plan_sparse_factor": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P, _P, _P]),
    "ras_plan_sparse_schedule": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32), _P, _P,
                                           _P, _P]),
    "ras_plan_sparse_lanes": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int64), _P, _P,
                                        _P]),
    "ras_sparse_max_rows": (C.c_int64, [C.c_int32]),
    "ras_plan_destroy": (None, [_P]),
    "ras_setup": (C.c_int, [C.POINTER(CSRStruct), C.POINTER(PartitionStruct), C.c_int32, C.POINTER(LocalStruct),
                            _P, C.POINTER(_P)]),
    "ras_setup_from_plan": (C.c_int, [_P, _P, C.POINTER(_P)]),
    "ras_handle_get_stats": (C.c_int, [_P, C.POINTER(PlanStats)]),
    "ras_solve": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "ras_solve_noalloc": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "ras_batch_solve": (C.c_int, [C.c_int32, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(C.c_int32),
                                  C.POINTER(SolveOpts), C.POINTER(SolveInfo)]),
    "ras_residual_history": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "ras_local_solve_counts": (C.c_int, [_P, C.c_int32, _P]),
    "ras_partition_sets": (C.c_int, [_P, _P, _P, _P]),
    "ras_relative_residual": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double)]),
    "ras_handle_factor": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "ras_phase_seconds": (C.c_int, [_P, C.c_int32, _P]),
    "ras_autotune": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "ras_destroy": (None, [_P]),
    "ras_pause": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "ras_cancel": (C.c_int, [_P]),
    "ras_server_create": (C.c_int, [C.c_int64, C.c_double, _P, C.POINTER(_P)]),
    "ras_server_submit": (C.c_int, [_P, C.POINTER(CSRStruct), C.POINTER(PartitionStruct), C.c_int32,
                                    C.POINTER(LocalStruct), _P, C.c_int32, C.c_double, C.POINTER(C.c_uint64)]),
    "ras_server_poll": (C.c_int, [_P, C.c_uint64, _P, _P, C.POINTER(C.c_double)]),
    "ras_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double]),
    "ras_server_get_stats": (C.c_int, [_P, _P]),
    "ras_server_destroy": (C.c_int, [_P]),
    "ras_async_next_step": (C.c_int32, [C.c_int32, C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_double,
                                        C.c_double, C.c_int32]),
    "ras_final_status": (C.c_int, [C.c_int32]),
    "ras_last_error": (C.c_char_p, []),
    "ras_version": (C.c_char_p, []),
}

_lib_handle = None


class RasError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib() -> C.CDLL:
    """The loaded native library; raises if it has not been built."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"native library missing: {LIB_PATH} (build it with python -m paper_2003_05361_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib_handle = L
    return _lib_handle


def _check(st: int, allow=(RAS_OK,)) -> int:
    if st not in allow:
        raise RasError(st, lib().ras_last_error().decode())
    return st


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ----------------------------------------------------------------------------- descriptions
def partition(kind: str, parts, grid=(1, 1, 1), seed: int = 0, jitter: float = 0.0, owner=None) -> dict:
    """Partition description (Sec. 3.2.1): kind in regular_1d / regular_2d / regular_3d / rcb / explicit."""
    if kind not in PART_KINDS:
        raise ValueError(kind)
    parts = tuple(parts) if isinstance(parts, (tuple, list)) else (int(parts),)
    return dict(kind=kind, parts=parts, grid=tuple(grid), seed=int(seed), jitter=float(jitter), owner=owner)


def local(kind: str = "chol", storage: str = "fp64", cg_iters: int = 0, robin_q=None) -> dict:
    """Local solver (Sec. 3.3.1): banded Cholesky ("chol"), nested-dissection sparse Cholesky
    ("chol_sparse") or fixed-k CG ("cg"); storage fp64/fp32/fp16.  robin_q in (0, 1]:
    Robin transmission (optimized RAS): the local matrices' diagonals are lowered by
    (1 - robin_q) times each row's coupling to points outside the subdomain; None: RAS."""
    if kind not in LOCAL_KINDS or storage not in STORAGES:
        raise ValueError((kind, storage))
    return dict(kind=kind, storage=storage, cg_iters=int(cg_iters), robin_q=robin_q)


class _Keep:
    """Host arrays that must stay alive while the C call runs."""

    def __init__(self):
        self.refs = []

    def add(self, a):
        self.refs.append(a)
        return a


def _csr(A, keep: _Keep) -> CSRStruct:
    if hasattr(A, "indptr") and hasattr(A, "indices"):
        indptr, indices, data = A.indptr, A.indices, A.data
        n = len(indptr) - 1
    else:
        raise TypeError("A must be a CSR matrix (scipy.sparse.csr_matrix or ras_inputs.CSR)")
    rp = keep.add(np.ascontiguousarray(indptr, dtype=np.int64))
    ci = keep.add(np.ascontiguousarray(indices, dtype=np.int32))
    va = keep.add(np.ascontiguousarray(data, dtype=np.float64))
    return CSRStruct(n, _ptr(rp, C.c_int64), _ptr(ci, C.c_int32), _ptr(va, C.c_double))


def _part(p: dict, A, keep: _Keep) -> PartitionStruct:
    s = PartitionStruct()
    s.kind = PART_KINDS[p["kind"]]
    grid = p.get("grid") or getattr(A, "grid", (1, 1, 1))
    if tuple(grid) == (1, 1, 1) and hasattr(A, "grid"):
        grid = A.grid
    g = (tuple(grid) + (1, 1, 1))[:3]
    s.grid[:] = [int(v) for v in g]
    parts = (tuple(p["parts"]) + (1, 1, 1))[:3]
    s.parts[:] = [int(v) for v in parts]
    s.seed = p.get("seed", 0)
    s.jitter = p.get("jitter", 0.0)
    if p.get("owner") is not None:
        o = keep.add(np.ascontiguousarray(p["owner"], dtype=np.int32))
        s.owner = _ptr(o, C.c_int32)
    return s


def _local(l: dict) -> LocalStruct:
    q = l.get("robin_q")
    return LocalStruct(LOCAL_KINDS[l["kind"]], int(l.get("cg_iters", 0)), STORAGES[l.get("storage", "fp64")],
                       0 if q is None else 1, 1.0 if q is None else float(q))


# ----------------------------------------------------------------------------- host-only plan
class Plan:
    """Host-side setup (no GPU): partition, overlap, local matrices, factors."""

    def __init__(self, A, part: dict, overlap: int, loc: dict):
        keep = _Keep()
        ptr = _P()
        _check(lib().ras_plan_create(C.byref(_csr(A, keep)), C.byref(_part(part, A, keep)), int(overlap),
                                     C.byref(_local(loc)), C.byref(ptr)))
        self._p = ptr
        self.n = len(A.indptr) - 1

    def stats(self) -> dict:
        s = PlanStats()
        _check(lib().ras_plan_get_stats(self._p, C.byref(s)))
        return s.as_dict()

    def sets(self):
        st = self.stats()
        owner = np.empty(self.n, dtype=np.int32)
        ptr = np.empty(st["parts"] + 1, dtype=np.int64)
        idx = np.empty(st["sum_local_rows"], dtype=np.int32)
        _check(lib().ras_plan_sets(self._p, owner.ctypes.data, ptr.ctypes.data, idx.ctypes.data))
        return owner, ptr, idx

    def comm_volume(self) -> np.ndarray:
        """P x P int64 matrix: [p, q] = values subdomain p reads from subdomain q's owned points per local solve."""
        P = self.stats()["parts"]
        v = np.empty((P, P), dtype=np.int64)
        _check(lib().ras_plan_comm_volume(self._p, v.ctypes.data))
        return v

    def band_width(self, p: int) -> int:
        """Lower half-bandwidth of subdomain p's local matrix."""
        w = C.c_int32()
        _check(lib().ras_plan_factor(self._p, p, None, C.byref(w)))
        return w.value

    def factor(self, p: int) -> tuple[np.ndarray, int]:
        w = C.c_int32()
        _check(lib().ras_plan_factor(self._p, p, None, C.byref(w)))
        owner, ptr, _ = self.sets()
        n = int(ptr[p + 1] - ptr[p])
        band = np.empty((n, w.value + 1))
        _check(lib().ras_plan_factor(self._p, p, band.ctypes.data, C.byref(w)))
        return band, w.value

    def sparse_factor(self, p: int):
        """(perm, row_ptr, col, val, diag) of subdomain p's sparse Cholesky factor:
        L L^T = A_p[perm][:, perm], L's strictly lower part in CSR, diag = L_kk."""
        nnz = C.c_int64()
        _check(lib().ras_plan_sparse_factor(self._p, p, None, None, None, None, None, C.byref(nnz)))
        _, ptr, _ = self.sets()
        n = int(ptr[p + 1] - ptr[p])
        perm = np.empty(n, dtype=np.int32)
        rp = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz.value, dtype=np.int32)
        val = np.empty(nnz.value)
        diag = np.empty(n)
        _check(lib().ras_plan_sparse_factor(self._p, p, perm.ctypes.data, rp.ctypes.data, col.ctypes.data,
                                            val.ctypes.data, diag.ctypes.data, C.byref(nnz)))
        return perm, rp, col, val, diag

    def sparse_schedule(self, p: int, pass_: int) -> dict:
        """Solve schedule of subdomain p's sparse factor for one pass (0: L, 1: L^T):
        step_ptr, meta (records x 4: slot written, first entry, end, 0), col, val,
        slots (block slots beyond n) and min_block."""
        ns, nr, ne = C.c_int32(), C.c_int64(), C.c_int64()
        sl, mb = C.c_int32(), C.c_int32()
        _check(lib().ras_plan_sparse_schedule(self._p, p, pass_, C.byref(ns), C.byref(nr), C.byref(ne), C.byref(sl),
                                              C.byref(mb), None, None, None, None))
        step = np.empty(ns.value + 1, dtype=np.int32)
        meta = np.empty((nr.value, 4), dtype=np.int32)
        col = np.empty(ne.value, dtype=np.int32)
        val = np.empty(ne.value)
        _check(lib().ras_plan_sparse_schedule(self._p, p, pass_, None, None, None, None, None, step.ctypes.data,
                                              meta.ctypes.data, col.ctypes.data, val.ctypes.data))
        return {"step_ptr": step, "meta": meta, "col": col, "val": val, "slots": sl.value, "min_block": mb.value}

    def sparse_lanes(self, p: int, pass_: int) -> dict:
        """The same pass in the device's lane layout: wave (waves x 2: first round,
        rounds), col and val (rounds x 64 items)."""
        nw, ni = C.c_int32(), C.c_int64()
        _check(lib().ras_plan_sparse_lanes(self._p, p, pass_, C.byref(nw), C.byref(ni), None, None, None))
        wave = np.empty((nw.value, 2), dtype=np.int32)
        col = np.empty(ni.value, dtype=np.int32)
        val = np.empty(ni.value)
        _check(lib().ras_plan_sparse_lanes(self._p, p, pass_, None, None, wave.ctypes.data, col.ctypes.data,
                                           val.ctypes.data))
        return {"wave": wave, "col": col.reshape(-1, 64), "val": val.reshape(-1, 64)}

    def factor_fp16(self, p: int) -> tuple[np.ndarray, np.ndarray]:
        band, w = self.factor(p)
        bits = np.empty(band.shape, dtype=np.uint16)
        scale = np.empty(band.shape[0], dtype=np.float32)
        _check(lib().ras_plan_factor_fp16(self._p, p, bits.ctypes.data, scale.ctypes.data))
        return bits, scale

    def setup(self, stream=None) -> "Handle":
        h = _P()
        sp = _stream_ptr(stream)
        _check(lib().ras_setup_from_plan(self._p, sp, C.byref(h)))
        return Handle(h, self.n, sp)

    def close(self):
        if getattr(self, "_p", None) and _lib_handle is not None:
            try:
                _lib_handle.ras_plan_destroy(self._p)
            except Exception:
                pass
            self._p = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime (or a profiler's tool library)
        # may already be gone: leave the memory to the process exit then
        if not _finalizing():
            self.close()


# ----------------------------------------------------------------------------- device handle
def _stream_ptr(stream):
    if stream is None:
        import torch

        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(getattr(stream, "cuda_stream", stream))


def _order_before(stream_value: int):
    """Wait on the host for torch's current stream unless it is the library's
    stream (the library's calls block until their results are on the device,
    so nothing is needed afterwards)."""
    import torch

    cur = torch.cuda.current_stream()
    if (cur.cuda_stream or 0) != stream_value:
        cur.synchronize()


def _rhs(b, n: int, what: str = "b"):
    """b as the C ABI takes it: a contiguous float64 CUDA tensor of shape [n] or
    [nrhs, n] (nrhs >= 1).  The library reads nrhs * n values from its address,
    so a wrong shape is refused here, before any launch."""
    import torch

    if not isinstance(b, torch.Tensor) or b.device.type != "cuda" or b.dtype != torch.float64:
        raise TypeError(f"{what} must be a float64 CUDA tensor")
    if b.dim() not in (1, 2) or b.shape[-1] != n or b.numel() == 0:
        raise ValueError(f"{what} must have shape [{n}] or [nrhs >= 1, {n}], got {tuple(b.shape)}")
    return b.contiguous()


def _initial(x0, b, what: str = "x0"):
    """A writable copy of the initial guess on b's device (zeros if x0 is None)."""
    import torch

    if x0 is None:
        return torch.zeros_like(b)
    if not isinstance(x0, torch.Tensor) or tuple(x0.shape) != tuple(b.shape):
        raise ValueError(f"{what} must be a tensor of b's shape {tuple(b.shape)}")
    return x0.to(device=b.device, dtype=torch.float64).contiguous().clone()


def _opts(tol, mode, max_sweeps, max_seconds, detect, workgroups, team=0, pace=None,
          detect_factor=1.0) -> SolveOpts:
    return SolveOpts(MODES[mode], DETECT[detect], float(tol), int(max_sweeps), float(max_seconds), int(workgroups),
                     int(team), float(DEFAULT_PACE if pace is None else pace), float(detect_factor))


class Handle:
    """A system set up on the device (Alg. 1's INITIALIZATION_AND_SETUP done)."""

    def __init__(self, ptr, n: int, stream):
        self._h = ptr
        self.n = n
        self.last_nrhs = 0
        self._stream = stream.value or 0  # the HIP stream the library uses for this handle

    def _order_after_current_stream(self):
        """The library reads b and x on the handle's stream; tensors made (or
        written) on torch's current stream must be complete before that."""
        _order_before(self._stream)

    def stats(self) -> dict:
        s = PlanStats()
        _check(lib().ras_handle_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def solve(self, b, x0=None, tol: float = 1e-8, mode: str = "async", max_sweeps: int = 1_000_000,
              max_seconds: float = 0.0, detect: str = "central", workgroups: int = 0, team: int = 0,
              allow_unconverged=True, pace=None, noalloc: bool = False, detect_factor: float = 1.0):
        """Solve A x = b on the device.  b: float64 CUDA tensor [n] or [nrhs, n].
        mode: "sync", "async" or "ordered"; detect: "central", "decentral" or
        "estimate" (a library option: stop on the owned-residual estimate once every
        subdomain has updated, verified exactly like the others);
        pace (async): neighbour wait budget before a read, in units of the
        previous update's time (None: the library's choice per local solver).
        detect_factor (async, ordered): the detector tests detect_factor * tol, the
        verification tol (> 1: stops that fail verification and resume).
        noalloc: run through ras_solve_noalloc (workspace in the library's fixed
        device scratch of NOALLOC_SCRATCH_BYTES; x is still allocated here unless
        x0 is given).  Returns (x, infos) with x the same shape as b."""
        b = _rhs(b, self.n)
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        x = _initial(x0, b)
        infos = (SolveInfo * nrhs)()
        self._order_after_current_stream()
        fn = lib().ras_solve_noalloc if noalloc else lib().ras_solve
        st = fn(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), nrhs,
                C.byref(_opts(tol, mode, max_sweeps, max_seconds, detect, workgroups, team, pace, detect_factor)),
                infos)
        _check(st, (RAS_OK, RAS_NOT_CONVERGED) if allow_unconverged else (RAS_OK,))
        self.last_nrhs = nrhs
        return x, [i.as_dict() for i in infos]

    def residual_history(self, rhs: int = 0) -> tuple[np.ndarray, np.ndarray]:
        n = C.c_int64()
        _check(lib().ras_residual_history(self._h, rhs, None, None, 0, C.byref(n)))
        t = np.empty(n.value)
        r = np.empty(n.value)
        _check(lib().ras_residual_history(self._h, rhs, t.ctypes.data, r.ctypes.data, n.value, C.byref(n)))
        return t, r

    def local_solve_counts(self, rhs: int = 0) -> np.ndarray:
        c = np.empty(self.stats()["parts"], dtype=np.int64)
        _check(lib().ras_local_solve_counts(self._h, rhs, c.ctypes.data))
        return c

    PHASES = ("residual", "local_solve", "prolong", "other")

    def phase_seconds(self, rhs: int = 0) -> np.ndarray:
        """[P, 4] seconds of the last solve per subdomain in the phases PHASES
        (device wall clock)."""
        P = self.stats()["parts"]
        out = np.empty((P, 4))
        _check(lib().ras_phase_seconds(self._h, int(rhs), out.ctypes.data))
        return out

    def partition_sets(self):
        st = self.stats()
        owner = np.empty(self.n, dtype=np.int32)
        ptr = np.empty(st["parts"] + 1, dtype=np.int64)
        idx = np.empty(st["sum_local_rows"], dtype=np.int32)
        _check(lib().ras_partition_sets(self._h, owner.ctypes.data, ptr.ctypes.data, idx.ctypes.data))
        return owner, ptr, idx

    def autotune(self, b, sweeps: int = 20) -> tuple[int, float]:
        """Time `sweeps` synchronous sweeps for every feasible team size; keep the best.
        Returns (team, ms per sweep).  b: one right-hand side [n]."""
        import torch

        b = _rhs(b, self.n)
        if b.dim() != 1:
            raise ValueError("autotune takes one right-hand side of shape [n]")
        x = torch.zeros_like(b)
        t = C.c_int32()
        ms = C.c_double()
        self._order_after_current_stream()
        _check(lib().ras_autotune(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), int(sweeps),
                                  C.byref(t), C.byref(ms)))
        return t.value, ms.value

    def pause(self, p: int, paused: bool = True) -> None:
        """Stall (or resume) subdomain p of asynchronous solves; may be called from
        another thread while a solve runs.  Give paused solves a time limit."""
        _check(lib().ras_pause(self._h, int(p), 1 if paused else 0))

    def cancel(self) -> None:
        """Stop the asynchronous solve running on this handle (from another thread);
        it returns not converged with the current iterate."""
        _check(lib().ras_cancel(self._h))

    def factor(self, p: int) -> tuple[np.ndarray, int]:
        """Subdomain p's banded Cholesky factor as the solves use it (read back from
        the device): (band [n, w+1] float64, w), band[i, j - i + w] = L_ij."""
        w = C.c_int32()
        _check(lib().ras_handle_factor(self._h, int(p), None, C.byref(w)))
        owner, ptr, _ = self.partition_sets()
        n = int(ptr[p + 1] - ptr[p])
        band = np.empty((n, w.value + 1))
        _check(lib().ras_handle_factor(self._h, int(p), band.ctypes.data, C.byref(w)))
        return band, w.value

    def relative_residual(self, b, x) -> float:
        """||b - A x|| / ||b|| on the device (compensated); b and x of shape [n]."""
        b, x = _rhs(b, self.n), _rhs(x, self.n, "x")
        if b.dim() != 1 or x.dim() != 1 or x.device != b.device:
            raise ValueError("relative_residual takes b and x of shape [n] on one device")
        r = C.c_double()
        self._order_after_current_stream()
        _check(lib().ras_relative_residual(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                           C.byref(r)))
        return r.value

    def close(self):
        if getattr(self, "_h", None) and _lib_handle is not None:
            try:
                _lib_handle.ras_destroy(self._h)
            except Exception:
                pass
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime (or a profiler's tool library)
        # may already be gone: leave the memory to the process exit then
        if not _finalizing():
            self.close()


def setup(A, part: dict, overlap: int, loc: dict, stream=None) -> Handle:
    keep = _Keep()
    h = _P()
    sp = _stream_ptr(stream)
    _check(lib().ras_setup(C.byref(_csr(A, keep)), C.byref(_part(part, A, keep)), int(overlap),
                           C.byref(_local(loc)), sp, C.byref(h)))
    return Handle(h, len(A.indptr) - 1, sp)


def batch_solve(handles: Sequence[Handle], bs, xs=None, tol: float = 1e-8, mode: str = "async",
                max_sweeps: int = 1_000_000, max_seconds: float = 0.0, detect: str = "central", workgroups: int = 0,
                team: int = 0, pace=None, detect_factor: float = 1.0):
    """Solve several systems in one persistent launch (same local solver kind/storage)."""
    import torch

    m = len(handles)
    if len(bs) != m or (xs is not None and len(xs) != m):
        raise ValueError("one right-hand side (and one x, if given) per handle")
    bs = [_rhs(b, h.n, f"bs[{i}]") for i, (h, b) in enumerate(zip(handles, bs))]
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    else:
        for i, (x, b) in enumerate(zip(xs, bs)):
            if not isinstance(x, torch.Tensor) or tuple(x.shape) != tuple(b.shape) or x.device != b.device \
                    or x.dtype != torch.float64:
                raise ValueError(f"xs[{i}] must be a float64 tensor of bs[{i}]'s shape on its device")
        xs = [x.contiguous() for x in xs]
    nr = [1 if b.dim() == 1 else b.shape[0] for b in bs]
    H = (_P * m)(*[h._h for h in handles])
    B = (_P * m)(*[b.data_ptr() for b in bs])
    X = (_P * m)(*[x.data_ptr() for x in xs])
    NR = (C.c_int32 * m)(*nr)
    infos = (SolveInfo * sum(nr))()
    for h in handles:
        h._order_after_current_stream()
    st = lib().ras_batch_solve(m, H, B, X, NR,
                               C.byref(_opts(tol, mode, max_sweeps, max_seconds, detect, workgroups, team, pace,
                                             detect_factor)), infos)
    _check(st, (RAS_OK, RAS_NOT_CONVERGED))
    out, k = [], 0
    for r in nr:
        out.append([infos[k + j].as_dict() for j in range(r)])
        k += r
    return xs, out


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64), ("active", C.c_int64),
                ("slices", C.c_int64), ("in_use_bytes", C.c_int64), ("peak_in_use_bytes", C.c_int64),
                ("budget_bytes", C.c_int64), ("device_seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """Continuous-batching solver service (the library's native server): systems
    are admitted while their device memory fits the budget and advanced together
    in time-sliced batched asynchronous launches."""

    def __init__(self, hbm_budget_bytes: int, slice_seconds: float = 0.02, stream=None):
        p = _P()
        st = None if stream is None else _stream_ptr(stream)
        _check(lib().ras_server_create(int(hbm_budget_bytes), float(slice_seconds), st, C.byref(p)))
        self._s = p
        self._shapes = {}  # ticket -> (n, nrhs): the size of the result poll receives

    def submit(self, A, part: dict, overlap: int, loc: dict, B, tol: float = 1e-8) -> int:
        """Queue a system; B is a host array [n] or [nrhs, n].  Returns a ticket."""
        keep = _Keep()
        Bh = keep.add(np.ascontiguousarray(B, dtype=np.float64))
        n = len(A.indptr) - 1
        if Bh.ndim not in (1, 2) or Bh.shape[-1] != n or Bh.size == 0:
            raise ValueError(f"B must have shape [{n}] or [nrhs >= 1, {n}], got {Bh.shape}")
        nrhs = 1 if Bh.ndim == 1 else Bh.shape[0]
        t = C.c_uint64()
        _check(lib().ras_server_submit(self._s, C.byref(_csr(A, keep)), C.byref(_part(part, A, keep)), int(overlap),
                                       C.byref(_local(loc)), Bh.ctypes.data, nrhs, float(tol), C.byref(t)))
        self._shapes[t.value] = (n, nrhs)
        return t.value

    def poll(self, ticket: int, n: int, nrhs: int = 1):
        """(done, x[nrhs, n] or None, infos, latency_s); raises on a failed system.
        n and nrhs must be those of the submitted system (the library writes its
        whole solution into the array allocated here)."""
        if self._shapes.get(int(ticket), (n, nrhs)) != (n, nrhs):
            raise ValueError(f"ticket {ticket} is a system of (n, nrhs) = {self._shapes[int(ticket)]}")
        x = np.empty((nrhs, n))
        infos = (SolveInfo * nrhs)()
        lat = C.c_double()
        st = lib().ras_server_poll(self._s, int(ticket), x.ctypes.data, infos, C.byref(lat))
        if st == RAS_PENDING:
            return False, None, None, None
        self._shapes.pop(int(ticket), None)
        _check(st)
        return True, x, [i.as_dict() for i in infos], lat.value

    def wait(self, ticket: int, timeout: float = 60.0) -> bool:
        return lib().ras_server_wait(self._s, int(ticket), float(timeout)) == RAS_OK

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().ras_server_get_stats(self._s, C.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_s", None) and _lib_handle is not None:
            try:
                _lib_handle.ras_server_destroy(self._s)
            except Exception:
                pass
            self._s = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime (or a profiler's tool library)
        # may already be gone: leave the memory to the process exit then
        if not _finalizing():
            self.close()


def async_next_step(kernel_stop: str, verified_relres: float, tol: float, min_local_solves: int, max_sweeps: int,
                    elapsed_seconds: float = 0.0, max_seconds: float = 0.0, ordered: bool = False) -> str:
    """The library's decision after an asynchronous launch ends for one right-hand
    side: "converged", "resume", "diverged" or "limit" (host only)."""
    return STEPS[lib().ras_async_next_step(KSTOP[kernel_stop], float(verified_relres), float(tol),
                                           int(min_local_solves), int(max_sweeps), float(elapsed_seconds),
                                           float(max_seconds), int(bool(ordered)))]


def final_status(step: str) -> int:
    """The ras_solve status of a final step."""
    return int(lib().ras_final_status({v: k for k, v in STEPS.items()}[step]))


def sparse_max_rows(storage: str = "fp64") -> int:
    """Largest subdomain the sparse Cholesky solver accepts for a storage kind."""
    return int(lib().ras_sparse_max_rows(STORAGES[storage]))


def version() -> str:
    return lib().ras_version().decode()
