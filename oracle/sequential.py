"""O1: the plain sequential corrected BDF-k / CQ-BDF-k time stepper
(oracle; test infrastructure).

This is the result every WR sweep converges to: the solution {U^n} of the
time-stepping scheme is the unique fixed point of the iteration (Sec. 2.2
after eq. BDF-iter; Sec. 3.2 after eq. BDF-frac-iter).

Scheme (Sec. 2.1 eq. BDF for alpha = 1; Sec. 3.1 eqs. CQ-1 and BDF-frac for
0 < alpha < 1), with history U^n = v for n <= 0:
    tau^{-alpha} sum_{j=0..n} omega_j (U^{n-j} - v) + A U^n = fbar_n,  n = 1..N.
For BDF-k this equals tau^{-1} sum_{j=0..k} omega_j U^{n-j} because the
weights sum to zero and vanish beyond k; for CQ the subtraction of v is the
Caputo-to-Riemann-Liouville rewrite of Sec. 3.1.  Step n solves, as in the
cost paragraph of Sec. 3.2,
    (omega_0 I + tau^alpha A) U^n
        = sum_{j=1..n} omega_j (v - U^{n-j}) + omega_0 v + tau^alpha fbar_n.
Each step's linear system is solved by sparse LU followed by two steps of
iterative refinement whose residual is formed in long double, so every U^n is
the exact solution of its step rounded to FP64 (without refinement the LU's
error of order eps times the step matrix's condition number, ~5e3 on a
2047-point line with N = 2048, accumulates over the steps to ~4e-11).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bdf import corrected_source
from .cq import time_weights


def _as_sparse(A):
    return A if sp.issparse(A) else sp.csr_matrix(np.atleast_2d(np.asarray(A, dtype=np.float64)))


def source_terms(A, k, alpha, T, N, v, f=None, fder=None):
    """fbar_n, n = 1..N, as an [N, M] array (Sec. 2.1 eq. BDF / Table 1)."""
    A = _as_sparse(A)
    M = A.shape[0]
    v = np.asarray(v, dtype=np.float64).reshape(M)
    if f is None:
        f = np.zeros((N + 1, M))
    f = np.asarray(f, dtype=np.float64).reshape(N + 1, M)
    tau = T / N
    return corrected_source(k, tau, f, A @ v, fder)


def sequential(A, k, alpha, T, N, v, f=None, fder=None):
    """U^1..U^N of the corrected scheme as an [N, M] array.

    A    : [M, M] operator (sparse or dense), or a scalar mode eigenvalue
    v    : [M] initial value
    f    : [N+1, M] source at t_0..t_N, or None (f = 0)
    fder : [k-2, M] d^l f/dt^l (0), l = 1..k-2, or None (zero)
    """
    A = _as_sparse(A)
    M = A.shape[0]
    tau = T / N
    v = np.asarray(v, dtype=np.float64).reshape(M)
    w = time_weights(k, alpha, N + 1)
    fbar = source_terms(A, k, alpha, T, N, v, f, fder)
    S = sp.csc_matrix(w[0] * sp.identity(M) + tau ** alpha * A)
    lu = spla.splu(S)
    solve = refined_solver(lu, w[0], tau ** alpha, A)
    D = np.zeros((N + 1, M))          # D[n] = U^n - v, D[0] = 0
    U = np.zeros((N, M))
    for n in range(1, N + 1):
        # sum_{j=1..n} omega_j (v - U^{n-j}) = -sum_j omega_j D[n-j]
        hist = -(w[1:n + 1][::-1] @ D[:n]) if n > 0 else 0.0
        rhs = hist + w[0] * v + tau ** alpha * fbar[n - 1]
        U[n - 1] = solve(rhs)
        D[n] = U[n - 1] - v
    return U


def refined_solver(lu, c0, c1, A, mass=None, steps=2):
    """x = (c0 E + c1 A)^{-1} b with E = I (or the mass matrix): the LU solve
    plus `steps` refinement steps with the residual in long double."""
    A_ld = sp.csr_matrix(A, dtype=np.longdouble)
    E_ld = None if mass is None else sp.csr_matrix(mass, dtype=np.longdouble)
    c0_ld, c1_ld = np.longdouble(c0), np.longdouble(c1)

    def solve(b):
        x = lu.solve(b)
        b_ld = np.asarray(b, dtype=np.longdouble)
        for _ in range(steps):
            x_ld = x.astype(np.longdouble)
            ex = x_ld if E_ld is None else E_ld @ x_ld
            r = b_ld - (c0_ld * ex + c1_ld * (A_ld @ x_ld))
            x = x + lu.solve(r.astype(np.float64))
        return x
    return solve
