"""BDF-k weights and starting-step corrections (oracle; test infrastructure).

* Sec. 2.1, eq. (bdf-gen): delta_k(zeta) = sum_{l=1..k} (1 - zeta)^l / l
  = sum_{j=0..k} omega_j zeta^j.  The weights are returned as exact
  rationals by expanding each (1 - zeta)^l with the binomial theorem.
* Sec. 2.1, eq. (BDF) and Table 1: for 1 <= n <= k-1 the source of step n is
  corrected to
      fbar_n = f(t_n) + a_n (f(0) - A v) + sum_{l=1..k-2} b_{l,n} tau^l d^l f/dt^l (0),
  and a_n = b_{l,n} = 0 for n >= k.  The same correction is used by the
  CQ-BDF-k scheme (Sec. 3.1, eq. BDF-frac).
"""
from fractions import Fraction as Fr
from math import comb

import numpy as np


def bdf_weights(k):
    """omega_0..omega_k of BDF-k as exact Fractions (Sec. 2.1, eq. bdf-gen)."""
    if not 1 <= k <= 6:
        raise ValueError("BDF-k is defined here for k = 1..6")
    w = [Fr(0)] * (k + 1)
    for l in range(1, k + 1):
        for j in range(0, l + 1):
            w[j] += Fr(comb(l, j) * (-1) ** j, l)
    return w


# Table 1: a_n^{(k)}, n = 1..k-1, and b_{l,n}^{(k)}, l = 1..k-2, n = 1..k-1.
_A = {
    1: [],
    2: [Fr(1, 2)],
    3: [Fr(11, 12), Fr(-5, 12)],
    4: [Fr(31, 24), Fr(-7, 6), Fr(3, 8)],
    5: [Fr(1181, 720), Fr(-177, 80), Fr(341, 240), Fr(-251, 720)],
    6: [Fr(2837, 1440), Fr(-2543, 720), Fr(17, 5), Fr(-1201, 720), Fr(95, 288)],
}
_B = {
    1: [],
    2: [],
    3: [[Fr(1, 12), Fr(0)]],
    4: [[Fr(1, 6), Fr(-1, 12), Fr(0)],
        [Fr(0), Fr(0), Fr(0)]],
    5: [[Fr(59, 240), Fr(-29, 120), Fr(19, 240), Fr(0)],
        [Fr(1, 240), Fr(-1, 240), Fr(0), Fr(0)],
        [Fr(1, 720), Fr(0), Fr(0), Fr(0)]],
    6: [[Fr(77, 240), Fr(-7, 15), Fr(73, 240), Fr(-3, 40), Fr(0)],
        [Fr(1, 96), Fr(-1, 60), Fr(1, 160), Fr(0), Fr(0)],
        [Fr(-1, 360), Fr(1, 720), Fr(0), Fr(0), Fr(0)],
        [Fr(0), Fr(0), Fr(0), Fr(0), Fr(0)]],
}


def table1_a(k, n):
    """a_n^{(k)} of Table 1 (zero for n >= k)."""
    return _A[k][n - 1] if 1 <= n <= k - 1 else Fr(0)


def table1_b(k, l, n):
    """b_{l,n}^{(k)} of Table 1 (zero for n >= k or l outside 1..k-2)."""
    if 1 <= n <= k - 1 and 1 <= l <= k - 2:
        return _B[k][l - 1][n - 1]
    return Fr(0)


def corrected_source(k, tau, f, Av, fder):
    """fbar_n for n = 1..N (Sec. 2.1 eq. BDF; Sec. 3.1 eq. BDF-frac).

    f    : array [N+1, M], f(t_0) .. f(t_N)  (t_n = n tau)
    Av   : array [M], A applied to the initial value v
    fder : array [k-2, M] with d^l f/dt^l (0), l = 1..k-2, or None (zero)
    Returns fbar as array [N, M] (row n-1 holds fbar_n).
    """
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[0] - 1
    fbar = f[1:].copy()
    for n in range(1, min(k - 1, N) + 1):
        fbar[n - 1] += float(table1_a(k, n)) * (f[0] - Av)
        if fder is not None:
            for l in range(1, k - 1):
                fbar[n - 1] += float(table1_b(k, l, n)) * tau ** l * fder[l - 1]
    return fbar
