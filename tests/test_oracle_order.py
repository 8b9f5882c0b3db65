"""PIN-9: the corrected BDF-k / CQ-BDF-k schemes of the oracle converge with
order k against exact single-mode solutions (Lemma 2.2 eq. err-BDF; Lemma 3.2
eq. err-BDF-frac).  This pins the weights and every row of Table 1 that the
forcing activates; a planted wrong Table 1 entry breaks it."""
import numpy as np
import pytest

import oracle.bdf as bdf
from oracle.exact import heat_trig_mode, subdiffusion_half_mode
from oracle.sequential import sequential


def _heat_slope(k, T=10.0, mu=0.5, Ns=(400, 800)):
    # f = cos t + sin t, v = 0: f(0) - A v = 1 and d^l f/dt^l (0) = 1, -1, -1, 1 (l = 1..4),
    # so every a_n and b_{l,n} of Table 1 enters.  The error is read at t = T: the bound of
    # Lemma 2.2 is O(tau^k) at fixed t_n, and the horizon T = 10 keeps BDF6's parasitic
    # roots (modulus ~0.86 per step) far below the measured error.
    errs = []
    for N in Ns:
        t = T * np.arange(N + 1) / N
        fd = np.array([[1.0], [-1.0], [-1.0], [1.0]])[:k - 2] if k > 2 else None
        f = (np.cos(t) + np.sin(t))[:, None]
        U = sequential(np.array([[mu]]), k, 1.0, T, N, np.array([0.0]), f, fd)
        errs.append(abs(U[-1, 0] - heat_trig_mode(mu, 0.0, T)))
    return np.log2(errs[0] / errs[1])


@pytest.mark.parametrize("k", range(1, 7))
def test_heat_order(k):
    assert abs(_heat_slope(k) - k) <= 0.15


@pytest.mark.parametrize("k,Ns", [(1, (80, 160)), (2, (80, 160)), (3, (80, 160)), (4, (80, 160)),
                                  (5, (160, 320))])
def test_subdiffusion_half_order(k, Ns):
    # alpha = 1/2, f = 0: exact mode E_{1/2}(-mu t^{1/2}) = erfcx(mu sqrt t).  CQ-BDF6's
    # measurable window is swamped by its parasitic initial layer and then by roundoff in
    # FP64; its Table 1 row is pinned by the heat test and its weights by the Cauchy test.
    T, mu = 1.0, 3.0
    errs = []
    for N in Ns:
        U = sequential(np.array([[mu]]), k, 0.5, T, N, np.array([1.0]))
        errs.append(abs(U[-1, 0] - subdiffusion_half_mode(mu, 1.0, T)))
    assert abs(np.log2(errs[0] / errs[1]) - k) <= 0.3


@pytest.mark.parametrize("k,which", [(2, ("a", 1)), (3, ("a", 1)), (4, ("a", 2)), (5, ("b", 2, 1)),
                                     (5, ("b", 3, 1)), (6, ("b", 1, 3)), (6, ("a", 5)), (4, ("b", 1, 2))])
def test_planted_table1_mistake_breaks_order(monkeypatch, k, which):
    # A plausible typo in one Table 1 entry must be caught by the order test above.
    from fractions import Fraction
    A = {kk: list(v) for kk, v in bdf._A.items()}
    B = {kk: [list(r) for r in v] for kk, v in bdf._B.items()}
    if which[0] == "a":
        A[k][which[1] - 1] += Fraction(1, 10)
    else:
        B[k][which[1] - 1][which[2] - 1] += Fraction(1, 10)
    monkeypatch.setattr(bdf, "_A", A)
    monkeypatch.setattr(bdf, "_B", B)
    assert abs(_heat_slope(k) - k) > 0.15
