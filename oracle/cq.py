"""Convolution-quadrature BDF-k weights (oracle; test infrastructure).

Sec. 3.1, eqs. (CQ) and (delta): the weights omega_j^{(alpha)} are the
power-series coefficients of delta_k(xi)^alpha, with delta_k the BDF-k
generating polynomial of eq. (bdf-gen).  The paper notes they can be
obtained by FFT or by a recursion; this module uses the recursion for the
power of a power series (J.C.P. Miller; Knuth, TAOCP vol. 2, Sec. 4.7):
if P = sum p_i xi^i with p_0 != 0 and Q = P^alpha = sum c_j xi^j, then
comparing coefficients in P Q' = alpha P' Q gives
    c_0 = p_0^alpha,
    c_j = 1/(j p_0) * sum_{i=1..min(j,k)} ((alpha + 1) i - j) p_i c_{j-i}.
For alpha = 1 the recursion returns the BDF weights followed by zeros.
"""
import numpy as np

from .bdf import bdf_weights


def cq_weights(k, alpha, n):
    """omega_0^{(alpha)} .. omega_{n-1}^{(alpha)} in FP64 (Sec. 3.1, eq. delta)."""
    if not 0.0 < alpha <= 1.0:
        raise ValueError("alpha must lie in (0, 1]")
    p = [float(x) for x in bdf_weights(k)]
    c = np.zeros(n, dtype=np.float64)
    if n == 0:
        return c
    c[0] = p[0] ** alpha
    for j in range(1, n):
        acc = 0.0
        for i in range(1, min(j, k) + 1):
            acc += ((alpha + 1.0) * i - j) * p[i] * c[j - i]
        c[j] = acc / (j * p[0])
    return c


def time_weights(k, alpha, N):
    """The N weights omega_0..omega_{N-1} that enter the N-step scheme.

    alpha == 1: the BDF-k weights (zero beyond index k); otherwise the CQ
    weights.  Both schemes share the form tau^{-alpha} sum_j omega_j U^{n-j}.
    """
    w = np.zeros(N, dtype=np.float64)
    if alpha == 1.0:
        b = [float(x) for x in bdf_weights(k)]
        m = min(N, k + 1)
        w[:m] = b[:m]
        return w
    return cq_weights(k, alpha, N)
