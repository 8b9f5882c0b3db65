"""O3: one WR sweep as a single dense space-time solve (oracle; test
infrastructure, tiny grids only).

Builds the kappa-circulant matrix B_k(kappa) entry by entry from its
definition (Sec. 2.2 after eq. BDF-k-F; Sec. 3.2 after eq. BDF-subdiff-F),
the all-at-once matrix P = tau^{-alpha} (B (x) I_M) + (I_N (x) A) of eqs.
BDF-k-matrix / BDF-k-matrix-frac, and solves P U_m = F_{m-1} with LAPACK.
No FFT, no diagonalization.
"""
import numpy as np

from .cq import time_weights


def kappa_circulant(k, alpha, N, kappa):
    """Dense B_k(kappa) (N x N)."""
    w = time_weights(k, alpha, N)
    B = np.zeros((N, N))
    for n in range(N):
        for j in range(N):
            B[n, j] = w[n - j] if n >= j else kappa * w[N + n - j]
    return B


def lower_toeplitz(k, alpha, N):
    """The lower-triangular part L of B (the sequential scheme's matrix)."""
    w = time_weights(k, alpha, N)
    L = np.zeros((N, N))
    for n in range(N):
        for j in range(n + 1):
            L[n, j] = w[n - j]
    return L


def all_at_once(A, k, alpha, T, N, kappa, mass=None):
    """Dense P (NM x NM), time index slowest.  With a mass matrix (P1 finite
    elements) the time part is B (x) mass instead of B (x) I."""
    A = np.asarray(A.toarray() if hasattr(A, "toarray") else A, dtype=np.float64)
    M = A.shape[0]
    tau = T / N
    E = np.eye(M) if mass is None else np.asarray(mass.toarray() if hasattr(mass, "toarray") else mass)
    return tau ** (-alpha) * np.kron(kappa_circulant(k, alpha, N, kappa), E) + np.kron(np.eye(N), A)


def sweep_dense(A, k, alpha, T, N, kappa, F, mass=None):
    """U_m = P^{-1} F_{m-1} by one dense LU solve; F is [N, M]."""
    P = all_at_once(A, k, alpha, T, N, kappa, mass)
    F = np.asarray(F, dtype=np.float64)
    return np.linalg.solve(P, F.reshape(-1)).reshape(F.shape)
