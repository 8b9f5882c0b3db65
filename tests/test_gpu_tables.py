"""The paper's worked examples through the C ABI on the GPU: Sec. 4 Example 1
(Table 2, heat, Algorithm 1) and Example 2 (Table 3, subdiffusion alpha = 1/2,
Algorithm 2), 1D, h = 1/1000 (m = 999, so the spatial solves take the
Bluestein sine transform), N = 100 (a time axis that is not a power of two, so
the sweep takes the Bluestein time DFTs), the direct form from U_0 = 0, FP64.
The error after each sweep m, e_m^N = ||U_m^N - U^N||_{L2(Omega)} against the
sequential oracle, must reproduce the printed rows m = 0..3 for every k (rows
4-5 are at the paper's roundoff floor)."""
import os

import numpy as np
import pytest

from oracle.grid import Grid, l2h
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import gpu_iterates, oracle_solution

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([float(x) for x in line.split()[1:]])
    return np.array(rows)


def _printed_match(got, printed):
    # within one unit of the last printed digit (plus the rounding half-unit)
    unit = 10.0 ** (np.floor(np.log10(abs(printed))) - 2)
    return abs(got - printed) <= 1.5 * unit


def _errors(w):
    its, _ = gpu_iterates(w, 3, form="direct", init="zero")
    UN = oracle_solution(w)[-1]
    g = Grid(w.m)
    return [l2h(g, U[-1] - UN) for U in its]


@pytest.mark.parametrize("k", range(1, 7))
def test_table2_example1_on_gpu(k):
    printed = _golden("table2.txt")[:, k - 1]
    got = _errors(wl.example1(k))
    print(f"Table 2 k={k}: {['%.3g' % e for e in got]}", flush=True)
    for m in range(4):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])


@pytest.mark.parametrize("k", range(1, 7))
def test_table3_example2_on_gpu(k):
    # Row m = 3 (~1.3e-8) sits close to what the data can determine: the discrete
    # Dirac v puts terms of 7e9 into the Table 1 rows, and a one-ulp perturbation
    # of them moves e_3 by up to 0.4% (measured on the oracle).  Where that moves
    # it across a printed digit, row 3 is held to 2% of the printed value: the FD
    # oracle itself sits 0.9% from the paper's (P1 FEM) value there, plus that
    # sensitivity.
    printed = _golden("table3.txt")[:, k - 1]
    got = _errors(wl.example2(k))
    print(f"Table 3 k={k}: {['%.4g' % e for e in got]}", flush=True)
    for m in range(3):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])
    assert _printed_match(got[3], printed[3]) or abs(got[3] / printed[3] - 1) <= 0.02, (k, got[3])
