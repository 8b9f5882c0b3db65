"""Algorithm 3 (semilinear problems, Sec. 4) through the C ABI on the GPU:
Example 4 (Table 4: Allen-Cahn term, eps = 1, h = 1/1000, N = 100, kappa = 0.1,
inner stopping rule 1e-12) against the oracle's Algorithm 3 Newton step by
Newton step (the iterate after l steps, and the inner WR sweep count of each
step, which must also equal Table 4's), and a linear reaction term, where one
Newton step must reach the sequential oracle."""
import numpy as np
import pytest

from oracle.grid import Grid, l2h, laplacian
from oracle.nonlinear import algorithm3, nl_sequential
from oracle.sequential import sequential
from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, to_dev

pytestmark = pytest.mark.gpu


def _gpu_alg3(w, c3, c1, steps, tol=1e-12):
    import torch
    print(f"[gpu] algorithm 3 {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha} steps={steps}", flush=True)
    plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=tol, max_sweeps=40)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    st, inner, upd = B.pint_nonlinear_solve(plan.h, c3, c1, to_dev(w.v), to_dev(w.f), to_dev(w.fder), U, steps)
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    plan.close()
    return st, out, inner, upd


@pytest.mark.parametrize("alpha,k", [(0.25, 1), (0.25, 2), (0.75, 1), (0.75, 2), (0.75, 3)])
def test_example4_newton_steps_match_oracle(alpha, k):
    w, c3, c1 = wl.example4(k, alpha)
    A = laplacian(Grid(w.m))
    its, counts = algorithm3(A, k, alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder, c3, c1)
    UN = nl_sequential(A, k, alpha, w.T, w.N, w.v, w.f, w.fder, c3, c1)[-1]
    g = Grid(w.m)
    assert counts == [5, 4, 3]                                     # Table 4's inner counts
    for steps in (1, 2, 3):
        st, U, inner, upd = _gpu_alg3(w, c3, c1, steps)
        assert inner == counts[:steps], (inner, counts)
        err = errors(U, its[steps])
        print(f"alpha={alpha} k={k} l={steps}: inner={inner} max|W|={upd} (rel_l2, max_rel)={err} "
              f"e_l={l2h(g, U[-1] - UN):.3g}", flush=True)
        assert max(err) <= 1e-11, err
    assert l2h(g, U[-1] - UN) <= 1e-11                             # U_3 at the oracle's nonlinear solution


def test_linear_reaction_one_newton_step():
    w = wl.heat1d(seed=6, m=63, N=32, k=3, kappa=1e-2)
    w.alpha = 0.6
    c1 = 7.5
    import scipy.sparse as sp
    ref = sequential(laplacian(Grid(w.m)) + c1 * sp.identity(w.M), w.k, w.alpha, w.T, w.N, w.v, w.f, w.fder)
    st, U, inner, upd = _gpu_alg3(w, 0.0, c1, 2, tol=1e-13)
    assert max(errors(U, ref)) <= 1e-11
    assert upd[1] <= 1e-12 * np.max(np.abs(ref))
