"""Banded Cholesky factors computed on the device by ras_setup (Sec. 3.3.1: the
local factor is computed once, at setup) against the host factorisation of the
same plan (row-oriented, float64), read back through ras_handle_factor."""
import sys

import numpy as np
import pytest

import ras_inputs as R

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _ras():
    import paper_2003_05361_amd as ras

    ras.lib()
    return ras


CASES = [
    ("tpfa2d_56_3x2_g3", lambda: R.tpfa2d(np.exp(2.0 * R.gaussian_random_field_2d(56, 8.0, 4)), 10.0),
     ("regular_2d", (3, 2)), 3),
    ("laplace3d_20_2x2x1_g2_w141", lambda: R.laplace3d(20), ("regular_3d", (2, 2, 1)), 2),
    ("laplace3d_24_2x2x1_g2_w193_rowmajor", lambda: R.laplace3d(24), ("regular_3d", (2, 2, 1)), 2),
    ("laplace2d_7x5_strips6_tiny", lambda: R.laplace2d(7, 5), ("regular_1d", 6), 1),
]


@pytest.mark.parametrize("name,make,part,gamma", CASES, ids=[c[0] for c in CASES])
def test_device_factor_equals_host_factor_fp64(name, make, part, gamma):
    ras = _ras()
    _say(f"case: device factor fp64 {name}")
    A = make()
    spec = ras.partition(part[0], part[1], grid=A.grid)
    plan = ras.Plan(A, spec, gamma, ras.local("chol", "fp64"))
    h = ras.setup(A, spec, gamma, ras.local("chol", "fp64"))
    P = plan.stats()["parts"]
    for p in range(P):
        Lh, wh = plan.factor(p)
        Ld, wd = h.factor(p)
        assert wd == wh and Ld.shape == Lh.shape
        scale = np.abs(Lh).max()
        assert np.max(np.abs(Ld - Lh)) <= 1e-13 * scale, (p, np.max(np.abs(Ld - Lh)) / scale)
    h.close()
    plan.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_device_factor_storage_cast(storage):
    """FP32: each stored entry is float32(L_ij) of the device factor, within one float32
    ulp of float32 of the host factor.  FP16: entries are float16(L_ij / s_i) times the
    row scale s_i = float32(max_j |L_ij|); against the host quantisation, equal up to
    one float16 ulp of the row scale (the two float64 factors differ in the last bits)."""
    ras = _ras()
    _say(f"case: device factor {storage}")
    A = R.tpfa2d(np.exp(2.0 * R.gaussian_random_field_2d(56, 8.0, 4)), 10.0)
    spec = ras.partition("regular_2d", (3, 2), grid=A.grid)
    plan = ras.Plan(A, spec, 3, ras.local("chol", storage))
    h = ras.setup(A, spec, 3, ras.local("chol", storage))
    for p in range(plan.stats()["parts"]):
        Ld, w = h.factor(p)
        if storage == "fp32":
            # far and near entries are float32(L_ij); the triangle of each 32-row block is
            # stored inverted (the solver applies it as a product) and read back by
            # inverting again in float64, so it carries that round trip's rounding
            Lh, _ = plan.factor(p)
            off = Lh[:, :w].astype(np.float32).astype(np.float64)
            r = np.arange(Lh.shape[0])[:, None] % 32
            tri = np.arange(w)[None, :] >= w - r
            err = np.abs(Ld[:, :w] - off)
            assert np.all(err[~tri] <= 2.0 ** -23 * np.abs(off[~tri]) + 1e-300)
            rowmax = np.abs(Lh).max(axis=1, keepdims=True) * np.ones_like(off)
            assert np.all(err[tri] <= 1e-5 * rowmax[tri])
        else:
            bits, sc = plan.factor_fp16(p)
            deq = bits.view(np.float16).astype(np.float64) * sc.astype(np.float64)[:, None]
            ulp = 2.0 ** -10 * sc.astype(np.float64)[:, None]
            assert np.all(np.abs(Ld[:, :w] - deq[:, :w]) <= ulp), p
            # and nearly all entries are the same bits
            assert np.mean(Ld[:, :w] == deq[:, :w]) > 0.999
    h.close()
    plan.close()


def test_device_factor_reports_non_spd():
    ras = _ras()
    _say("case: device factor non-SPD")
    A = R.laplace2d(6).scipy().tolil()
    A[7, 7] = -4.0
    A = A.tocsr()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    with pytest.raises(ras.RasError) as e:
        ras.setup(A, ras.partition("regular_1d", 2), 1, ras.local("chol", "fp64"))
    assert e.value.status == -3
    assert "subdomain 0" in str(e.value) and "local row 7" in str(e.value)


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_host_and_device_layouts_give_the_same_iteration(storage, tol):
    """A handle set up from a host-factored plan (host layout, host block inverses) and
    one factored on the device iterate alike."""
    import torch

    ras = _ras()
    _say(f"case: host vs device layout {storage}")
    A = R.tpfa2d(np.exp(2.0 * R.gaussian_random_field_2d(64, 8.0, 4)), 10.0)
    spec = ras.partition("regular_2d", (2, 2), grid=A.grid)
    b = torch.tensor(R.uniform_rhs(A.n, 7), dtype=torch.float64, device="cuda")
    plan = ras.Plan(A, spec, 4, ras.local("chol", storage))
    hh = plan.setup()
    hd = ras.setup(A, spec, 4, ras.local("chol", storage))
    xh, _ = hh.solve(b, tol=0.0, mode="sync", max_sweeps=5)
    xd, _ = hd.solve(b, tol=0.0, mode="sync", max_sweeps=5)
    xh, xd = xh.cpu().numpy(), xd.cpu().numpy()
    assert np.max(np.abs(xh - xd)) <= tol * np.max(np.abs(xh))
    hh.close()
    hd.close()
    plan.close()
