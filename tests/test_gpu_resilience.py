"""Failure handling and restart on the GPU path, forced from the host: resume
from a saved iterate (INIT_USER) equals an uninterrupted solve bit for bit;
a NaN in the data is reported as PINT_E_DIVERGED; hitting max_sweeps returns
PINT_NOT_CONVERGED with the last iterate and its norms; the terminal-L2 stop
norm; argument errors on live plans."""
import numpy as np
import pytest
import torch

from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, oracle_solution, to_dev

pytestmark = pytest.mark.gpu


def _plan(w, **kw):
    return B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, **kw)


def test_resume_from_saved_iterate_is_bitwise_identical():
    w = wl.heat2d(seed=21, m=(31, 31), N=64, k=4, kappa=1e-3)
    v, f, fd = to_dev(w.v), to_dev(w.f), to_dev(w.fder)
    print("[gpu] resume test", flush=True)
    p = _plan(w)
    p.bind(v, f, fd)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    p.init_iterate(U)
    p.sweeps(U, 4)
    straight = U.cpu().numpy()
    p.init_iterate(U)
    p.sweeps(U, 2)
    saved = U.clone()                              # checkpoint after two sweeps
    p.close()
    q = _plan(w, init="user")                      # a new plan resumes from the checkpoint
    q.bind(v, f, fd)
    q.init_iterate(saved)                          # INIT_USER leaves it untouched
    q.sweeps(saved, 2)
    torch.cuda.synchronize()
    assert np.array_equal(saved.cpu().numpy(), straight)
    q.close()


def test_nan_in_data_reports_diverged():
    w = wl.heat1d(m=63, N=64)
    w.v[10] = np.nan
    p = _plan(w, tol=1e-12, max_sweeps=5)
    U, info = p.solve(to_dev(w.v), to_dev(w.f))
    assert info["status"] == B.PINT_E_DIVERGED
    assert info["sweeps"] == 1
    p.close()


def test_max_sweeps_returns_last_iterate_and_norms():
    w = wl.heat2d(seed=22, m=(15, 15), N=32, k=3, kappa=0.3)
    p = _plan(w, tol=1e-300, max_sweeps=3)
    U, info = p.solve(to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    assert info["status"] == B.PINT_NOT_CONVERGED and info["sweeps"] == 3
    assert len(info["upd"]) == 3 and info["upd"][2] < info["upd"][1] < info["upd"][0]
    # the returned iterate is the third sweep (compare with an explicit 3-sweep run)
    q = _plan(w)
    q.bind(to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    U3 = torch.empty_like(U)
    q.init_iterate(U3)
    q.sweeps(U3, 3)
    torch.cuda.synchronize()
    assert torch.equal(U, U3)
    p.close()
    q.close()


def test_terminal_l2_stop_norm():
    w = wl.heat1d(m=63, N=64, kappa=1e-2)
    p = _plan(w, tol=1e-13, max_sweeps=30, norm="l2T")
    U, info = p.solve(to_dev(w.v), to_dev(w.f))
    assert info["status"] == B.PINT_OK
    assert info["upd_l2T"][-1] <= 1e-13 < info["upd_l2T"][0]
    assert max(errors(U.cpu().numpy(), oracle_solution(w))) <= 1e-11
    p.close()


def test_errors_on_live_plan():
    w = wl.heat1d(m=63, N=64)
    p = _plan(w)
    U = torch.zeros((w.N, w.M), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PintError):
        p.sweeps(U, 1)                       # not bound yet
    with pytest.raises(B.PintError):
        B.pint_bind(p.h, None)               # v must not be NULL
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.PintError):
        B.pint_plan_set_workspace(p.h, small)
    p.close()
    # a plan without a workspace refuses to bind (nothing is allocated on the solve path)
    h = B.pint_plan_create(B.make_grid(w.m), B.make_params(w.k, w.alpha, w.T, w.N, w.kappa))
    with pytest.raises(B.PintError):
        B.pint_bind(h, torch.zeros(w.M, dtype=torch.float64, device="cuda"))
    B.pint_plan_destroy(h)
