"""pint_solve_noalloc (the solve for callers that cannot allocate device
memory: its workspace is a static device array) against pint_solve on the same
plan parameters and inputs, through the C ABI: two calls in a row, the second
with a smaller problem, and a plan whose workspace exceeds the array."""
import numpy as np
import pytest

from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, oracle_solution, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(plan, v, f, fder, U, max_sweeps):
    return B.pint_solve_noalloc(plan, v, f, fder, U, max_sweeps)


def _pair(w, precision, form="residual"):
    import torch
    print(f"[gpu] noalloc {w.name} m={w.m} N={w.N} {precision}/{form}", flush=True)
    v, f, fd = to_dev(w.v), to_dev(w.f), to_dev(w.fder)
    ref_plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-13, max_sweeps=30, precision=precision,
                      form=form)
    Uref, info = ref_plan.solve(v, f, fd)
    torch.cuda.synchronize()
    ref_plan.close()
    # a plan that never received a workspace
    h = B.pint_plan_create(B.make_grid(w.m), B.make_params(w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-13,
                                                           max_sweeps=30, precision=precision, form=form))
    U = torch.empty_like(Uref)
    st, upd, upd2, n = _noalloc(h, v, f, fd, U, 30)
    torch.cuda.synchronize()
    B.pint_plan_destroy(h)
    assert st == info["status"] == B.PINT_OK, (st, B.lib().pint_last_error())
    assert n == info["sweeps"] and upd == info["upd"] and upd2 == info["upd_l2T"]
    got = U.cpu().numpy()
    assert np.array_equal(got, Uref.cpu().numpy())            # same kernels, same inputs
    err = errors(got, oracle_solution(w))
    assert max(err) <= (1e-11 if precision == "fp64" else 1e-10), err


def test_noalloc_two_calls_second_smaller():
    _pair(wl.heat2d(seed=31, m=(63, 31), N=64, k=4, kappa=1e-3), "fp64")
    _pair(wl.heat1d(seed=32, m=100, N=32, k=3, kappa=1e-2), "mixed")


def test_noalloc_direct_form_after_residual():
    _pair(wl.heat2d(seed=33, m=(31, 31), N=32, k=3, kappa=1e-3), "fp64", form="direct")


def test_noalloc_rejects_plan_beyond_scratch():
    import torch
    w = wl.heat2d(m=(255, 255), N=512, k=4, kappa=1e-5)       # 269 MB of workspace > 64 MiB
    h = B.pint_plan_create(B.make_grid(w.m), B.make_params(w.k, w.alpha, w.T, w.N, w.kappa))
    U = torch.zeros((w.N, w.M), dtype=torch.float64, device="cuda")
    st, upd, _, n = _noalloc(h, to_dev(w.v), to_dev(w.f), to_dev(w.fder), U, 30)
    B.pint_plan_destroy(h)
    assert st == B.PINT_E_ARG and n == 0
    assert b"static scratch" in B.lib().pint_last_error()
    assert torch.count_nonzero(U).item() == 0
