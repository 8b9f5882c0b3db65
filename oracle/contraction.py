"""Contraction factor of the WR sweep for one spatial mode (oracle; test
infrastructure).

With A replaced by one eigenvalue mu (the reduction used in Sec. 2.2's
roundoff paragraph and in the proofs of Lemmas conv-heat and conv-frac), the
error e_m = U_m - U of the sweep obeys
    (tau^{-alpha} B_k(kappa) + mu I) e_m = kappa tau^{-alpha} Up e_{m-1},
where Up is the strictly upper part of B_k(kappa) divided by kappa.  The
asymptotic contraction per sweep is the spectral radius of
    J = kappa tau^{-alpha} (tau^{-alpha} B_k(kappa) + mu I)^{-1} Up.
For BDF1 this reduces to the Gander-Wu factor kappa R^N / (1 - kappa R^N),
R = 1/(1 + tau mu), quoted in Remark 2.3.
"""
import numpy as np

from .bruteforce import kappa_circulant
from .cq import time_weights


def iteration_matrix(k, alpha, T, N, kappa, mu):
    tau = T / N
    w = time_weights(k, alpha, N)
    B = kappa_circulant(k, alpha, N, kappa)
    Up = np.zeros((N, N))
    for n in range(N):
        for j in range(n + 1, N):
            Up[n, j] = w[N + n - j]
    P = tau ** (-alpha) * B + mu * np.eye(N)
    return kappa * tau ** (-alpha) * np.linalg.solve(P, Up)


def spectral_radius(k, alpha, T, N, kappa, mu):
    return float(np.max(np.abs(np.linalg.eigvals(iteration_matrix(k, alpha, T, N, kappa, mu)))))
