"""P1 finite elements (1D) on the GPU through the C ABI, against the FEM
oracle: converged trajectories (FP64 1e-11, mixed 1e-10, residual and direct
forms, BDF-k and CQ-BDF-k, time axes of every kind, grids whose sine length is
a power of two or not), each of the first three sweeps against Algorithm 1/2
with the mass matrix, and the paper's Examples 1-2 (Tables 2-3) in their P1
form."""
import os

import numpy as np
import pytest

from oracle.fem import l2_fe
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, gpu_iterates, gpu_solve, max_rel, oracle_iterates, oracle_solution

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# (m, N, k, alpha, kappa)
CASES = [
    (7, 16, 2, 1.0, 1e-2),
    (63, 64, 3, 1.0, 1e-3),      # sine length 128 (the power-of-two sine solve with the mass divide)
    (100, 32, 4, 0.5, 1e-3),
    (255, 100, 6, 1.0, 1e-3),    # time axis of 100 levels
    (40, 6, 5, 1.0, 0.1),
    (31, 2, 1, 1.0, 0.1),
    (1000, 64, 2, 0.7, 1e-3),
    (127, 1024, 3, 0.5, 1e-3),   # CQ history by the 2048-point convolution
    (9, 48, 1, 0.3, 1e-2),
    (2047, 2048, 2, 1.0, 1e-3),  # the largest line: one lane per dof in the residual
]


def _case(m, N, k, alpha, kappa):
    return wl.fem1d(seed=700 + m + N + k, m=m, N=N, k=k, alpha=alpha, kappa=kappa)


@pytest.mark.parametrize("m,N,k,alpha,kappa", CASES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fem_converged_matches_oracle(m, N, k, alpha, kappa, precision):
    w = _case(m, N, k, alpha, kappa)
    U, info = gpu_solve(w, precision=precision, tol=1e-14 if m <= 600 else 1e-12, max_sweeps=40)
    err = errors(U, oracle_solution(w))
    print(f"fem m={m} N={N} k={k} alpha={alpha} {precision}: sweeps={info['sweeps']} (rel_l2, max_rel)={err}",
          flush=True)
    assert max(err) <= (1e-11 if precision == "fp64" else 1e-10), (err, info)


@pytest.mark.parametrize("m,N,k,alpha,kappa", [c for c in CASES if c[4] >= 1e-3])
def test_fem_direct_form_matches_oracle(m, N, k, alpha, kappa):
    w = _case(m, N, k, alpha, kappa)
    U, info = gpu_solve(w, form="direct", tol=1e-12, max_sweeps=25)
    err = errors(U, oracle_solution(w))
    assert max(err) <= 1e-11, (err, info)


@pytest.mark.parametrize("m,N,k,alpha,kappa", [c for c in CASES if c[0] * c[1] <= 70000])
@pytest.mark.parametrize("form,init", [("residual", "v"), ("direct", "zero")])
def test_fem_each_sweep_matches_dense_dft_sweep(m, N, k, alpha, kappa, form, init):
    # The bound of the FD per-sweep test (transform rounding amplified by up to 1/kappa;
    # in the residual form the FP64 residual's rounding with a gain up to the condition
    # number of the spatial operator), the latter times 3 for the mass matrix, whose
    # eigenvalues lie in [1/3, 1].
    w = _case(m, N, k, alpha, kappa)
    got, norms = gpu_iterates(w, 3, form=form, init=init)
    ref = oracle_iterates(w, 3, form=form, init=init)
    mu = 4.0 * (m + 1) ** 2 * np.sin(np.pi * np.array([1, m]) / (2.0 * (m + 1))) ** 2
    cond = 3.0 * mu[1] / mu[0]
    bound = max(1e-12, 10 * EPS * np.log2(N) / kappa, EPS * cond if form == "residual" else 0.0)
    for s in range(1, 4):
        scale = max(np.linalg.norm(ref[s]), 1e-300)
        assert np.linalg.norm(got[s] - ref[s]) / scale <= bound, (s, np.linalg.norm(got[s] - ref[s]) / scale)
        assert max_rel(got[s], ref[s]) <= bound, (s, max_rel(got[s], ref[s]))


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(x) for x in line.split()[1:]])
    return np.array(rows)


def _printed_match(got, printed):
    unit = 10.0 ** (np.floor(np.log10(abs(printed))) - 2)
    return abs(got - printed) <= 1.5 * unit


def _fem_errors(w):
    its, _ = gpu_iterates(w, 3, form="direct", init="zero")
    UN = oracle_solution(w)[-1]
    return [l2_fe(w.m[0], U[-1] - UN) for U in its]


@pytest.mark.parametrize("k", range(1, 7))
def test_fem_table2_example1_on_gpu(k):
    printed = _golden("table2.txt")[:, k - 1]
    got = _fem_errors(wl.example1_fem(k))
    print(f"P1 Table 2 k={k}: {['%.4g' % e for e in got]}", flush=True)
    for m in range(4):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])


@pytest.mark.parametrize("k", range(1, 7))
def test_fem_table3_example2_on_gpu(k):
    # Rows 0..2 to the printed digits; row 3 likewise for k <= 3.  For k >= 4 row 3
    # (~1.3e-8) is near the rounding floor of any transform-based sweep on this data:
    # the L2-projected Dirac puts entries of ~1e9 into the Table 1 rows (k - 1 of them),
    # and rounding noise of one ulp of the largest spectrum entry (times log2 N) added to
    # the oracle's Step 1 moves its e_3 anywhere in 3e-9 .. 6e-8 (measured on the CPU);
    # there row 3 is held to 5% of the printed value.
    printed = _golden("table3.txt")[:, k - 1]
    got = _fem_errors(wl.example2_fem(k))
    print(f"P1 Table 3 k={k}: {['%.4g' % e for e in got]}", flush=True)
    for m in range(3 if k >= 4 else 4):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])
    assert abs(got[3] - printed[3]) <= 0.05 * printed[3], (k, got[3], printed[3])


def test_fem_rejects_tridiagonal_knob_and_unsupported_solvers():
    import torch

    from paper_2007_13125_amd import binding as B
    from tests.gpu_util import to_dev
    w = _case(63, 64, 2, 1.0, 1e-3)
    plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, space="fem")
    with pytest.raises(B.PintError):
        plan.set_variants([0, 0, 0, 1])
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    with pytest.raises(B.PintError):
        B.pint_sequential_solve(plan.h, to_dev(w.v), to_dev(w.f), to_dev(w.fder), U)
    plan.close()
