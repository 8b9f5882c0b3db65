"""The windowed solve (sequential windows, WR sweeps inside each) through the C
ABI against the windowed oracle, and BDF1 windows against one global solve."""
import numpy as np
import pytest

from oracle.grid import Grid, laplacian
from oracle.windows import windowed_sequential
from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, oracle_solution, to_dev

pytestmark = pytest.mark.gpu


def _gpu_windows(w, nwin, N, fder=None, precision="fp64"):
    import torch
    print(f"[gpu] windows {w.name} m={w.m} nwin={nwin} N={N} k={w.k} alpha={w.alpha} {precision}", flush=True)
    plan = B.Plan(w.m, w.k, w.alpha, w.T / nwin, N, w.kappa, tol=1e-14, max_sweeps=40, precision=precision)
    U = torch.empty((nwin * N, w.M), dtype=torch.float64, device="cuda")
    st, upd, sw = B.pint_solve_windows(plan.h, nwin, to_dev(w.v), to_dev(w.f), to_dev(fder), U, 40)
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    plan.close()
    return st, out, sw


@pytest.mark.parametrize("dim,m,N,nwin,k,alpha,precision", [
    (1, (63,), 16, 4, 3, 1.0, "fp64"), (1, (100,), 20, 3, 2, 0.5, "fp64"), (2, (15, 7), 32, 3, 4, 1.0, "fp64"),
    (2, (31, 31), 16, 2, 2, 1.0, "mixed"), (3, (7, 5, 3), 8, 5, 1, 1.0, "fp64")])
def test_windows_match_windowed_oracle(dim, m, N, nwin, k, alpha, precision):
    mk = {1: lambda: wl.heat1d(seed=8, m=m[0], N=nwin * N, k=min(k, 2), T=1.0),
          2: lambda: wl.heat2d(seed=8, m=m, N=nwin * N, k=min(k, 2), T=1.0),
          3: lambda: wl.heat3d(seed=8, m=m, N=nwin * N, k=min(k, 2), T=1.0)}[dim]
    w = mk()
    w.k, w.alpha = k, alpha
    # derivatives of f at every window's start (zero: the recipe's f has none beyond
    # what the window sees); same on both sides
    fder = np.zeros((nwin, k - 2, w.M)) if k > 2 else None
    st, U, sw = _gpu_windows(w, nwin, N, fder, precision)
    ref = windowed_sequential(laplacian(Grid(w.m)), k, alpha, w.T / nwin, N, nwin, w.v, w.f, fder)
    err = errors(U, ref)
    assert st == B.PINT_OK and max(err) <= (1e-11 if precision == "fp64" else 1e-10), (err, sw)


def test_bdf1_windows_equal_global_solve():
    nwin, N = 4, 16
    w = wl.heat1d(seed=9, m=63, N=nwin * N, k=1, T=2.0)
    st, U, sw = _gpu_windows(w, nwin, N)
    assert max(errors(U, oracle_solution(w))) <= 1e-11
