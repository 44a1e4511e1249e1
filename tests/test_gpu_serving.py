"""Serving (continuous batching) through the C ABI on the GPU.

Checks: every admitted system retires with a verified residual below its
tolerance; the device-memory budget is never exceeded (the server's own peak
accounting); systems submitted while others run are admitted as memory frees
up; and a system's result is the same alone and in a mix, within the stated
tolerance (both runs asynchronous, so equal to tolerance, not bitwise):
||x_alone - x_mix|| / ||x_alone|| <= 1e-6 with both residuals < 1e-10.
"""
import time

import numpy as np
import pytest

import ras_inputs as R
from oracle import schwarz

pytestmark = pytest.mark.gpu


def _ras():
    import paper_2003_05361_amd as ras

    ras.lib()
    return ras


def _systems(seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(6):
        if k % 2 == 0:
            N = int(rng.integers(40, 90))
            A = R.tpfa2d(np.exp(rng.standard_normal((N, N))))
            part, loc = ("regular_2d", (2, 2)), ("chol", "fp32", 0)
        else:
            N = int(rng.integers(10, 16))
            A = R.tpfa3d(np.exp(rng.standard_normal((N, N, N))))
            part, loc = ("regular_3d", (2, 2, 2)), ("cg", "fp32", 8)
        nrhs = int(rng.integers(1, 4))
        B = rng.uniform(0, 1, (nrhs, A.n))
        out.append((A, part, loc, B))
    return out


def _submit(ras, srv, A, part, loc, B, tol):
    return srv.submit(A, ras.partition(part[0], part[1], grid=A.grid), 2, ras.local(*loc), B, tol)


def test_server_continuous_admission_and_budget():
    ras = _ras()
    print("case: server admission", flush=True)
    systems = _systems(1)
    budget = 48 << 20  # small enough that not every system fits at once
    srv = ras.Server(budget, slice_seconds=0.01)
    tickets = []
    for i, (A, part, loc, B) in enumerate(systems):
        tickets.append(_submit(ras, srv, A, part, loc, B, 1e-8))
        time.sleep(0.02 * (i % 3))  # arrivals while others are on the device
    for (A, part, loc, B), t in zip(systems, tickets):
        assert srv.wait(t, 120.0)
        done, x, infos, lat = srv.poll(t, A.n, B.shape[0])
        assert done and lat > 0
        for j in range(B.shape[0]):
            assert infos[j]["converged"]
            assert schwarz.relative_residual(A, x[j], B[j]) < 1e-8
    st = srv.stats()
    assert st["completed"] == len(systems) and st["active"] == 0 and st["queued"] == 0
    assert 0 < st["peak_in_use_bytes"] <= budget
    srv.close()


def test_server_result_same_alone_and_in_mix():
    ras = _ras()
    print("case: server alone vs mix", flush=True)
    systems = _systems(2)
    A, part, loc, B = systems[0]
    tol = 1e-10
    srv = ras.Server(8 << 30, slice_seconds=0.01)
    t = _submit(ras, srv, A, part, loc, B, tol)
    assert srv.wait(t, 120.0)
    _, x_alone, _, _ = srv.poll(t, A.n, B.shape[0])
    ts = [_submit(ras, srv, *s, tol) for s in systems]
    for s, tk in zip(systems, ts):
        assert srv.wait(tk, 120.0)
    _, x_mix, _, _ = srv.poll(ts[0], A.n, B.shape[0])
    for tk, s in zip(ts[1:], systems[1:]):
        srv.poll(tk, s[0].n, s[3].shape[0])
    for j in range(B.shape[0]):
        assert schwarz.relative_residual(A, x_alone[j], B[j]) < tol
        assert schwarz.relative_residual(A, x_mix[j], B[j]) < tol
        assert np.linalg.norm(x_alone[j] - x_mix[j]) <= 1e-6 * np.linalg.norm(x_alone[j])
    srv.close()


def test_server_rejects_oversized_system():
    ras = _ras()
    A = R.laplace2d(64)
    srv = ras.Server(1 << 16, slice_seconds=0.01)
    t = srv.submit(A, ras.partition("regular_2d", (2, 2), grid=A.grid), 2, ras.local("cg", "fp32", 4),
                   np.ones(A.n), 1e-8)
    assert srv.wait(t, 60.0)
    with pytest.raises(ras.RasError) as e:
        srv.poll(t, A.n)
    assert e.value.status == -4
    srv.close()
