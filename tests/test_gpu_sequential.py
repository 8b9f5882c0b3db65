"""The sequential-in-time GPU solver (the scheme stepped level by level, one
shifted spatial solve per step) against the sequential oracle: small shapes
entry by entry, and the 2D/3D heat workloads at full size on sampled dofs
against the per-sine-mode oracle."""
import numpy as np
import pytest

from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, oracle_modal, oracle_solution, to_dev

pytestmark = pytest.mark.gpu


def _seq(w):
    import torch
    print(f"[gpu] sequential {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha}", flush=True)
    plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    plan._data = (to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    B.pint_sequential_solve(plan.h, *plan._data, U)
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    plan.close()
    return out


CASES = [
    (1, (63,), 64, 2, 1.0), (1, (100,), 32, 6, 1.0), (1, (255,), 16, 3, 0.5), (1, (7,), 100, 4, 0.7),
    (2, (15, 7), 32, 4, 1.0), (2, (31, 31), 64, 3, 0.5), (2, (20, 13), 24, 5, 1.0),
    (3, (7, 15, 3), 16, 6, 1.0), (3, (6, 9, 5), 16, 2, 0.3),
]


@pytest.mark.parametrize("dim,m,N,k,alpha", CASES)
def test_sequential_matches_oracle(dim, m, N, k, alpha):
    mk = {1: lambda: wl.heat1d(seed=4, m=m[0], N=N, k=k), 2: lambda: wl.heat2d(seed=4, m=m, N=N, k=k),
          3: lambda: wl.heat3d(seed=4, m=m, N=N, k=k)}[dim]
    w = mk()
    w.alpha = alpha
    err = errors(_seq(w), oracle_solution(w))
    assert max(err) <= 1e-11, err


@pytest.mark.parametrize("name", ["heat2d", "heat3d"])
def test_sequential_full_size(name):
    w = getattr(wl, name)()
    U = _seq(w)
    dofs = np.random.default_rng(3).choice(w.M, 2048, replace=False)
    err = errors(U[:, dofs], oracle_modal(w, dofs))
    print(f"{name} sequential: (rel_l2, max_rel)={err}", flush=True)
    assert max(err) <= 1e-11, err
