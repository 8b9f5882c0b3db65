"""Semilinear extension: the modified Newton iteration with a time-averaged
Jacobian and inner waveform-relaxation sweeps (oracle; test infrastructure).

Problem (Sec. 4, extension to nonlinear problems, eq. fde-nonlinear):
    d_t^alpha u + A u + g(u) = f on (0, T],  u(0) = v,
here with the cubic g(u) = c3 u^3 + c1 u (Example 4, Allen-Cahn:
c3 = 1/eps^2, c1 = -1/eps^2), g'(u) = 3 c3 u^2 + c1.

Scheme (eq. BDF-CQ-m-r), with U^n = v for n <= 0:
    dbar^alpha U^n + A U^n + g(U^n) = fbar_n,  n = 1..N,
    dbar^alpha U^n = tau^{-alpha} sum_{j=0..n} omega_j (U^{n-j} - v),
    fbar_n = f(t_n) + a_n (f(0) - A v - g(v)) + sum_l b_{l,n} tau^l d^l f/dt^l (0).

nl_sequential: the scheme stepped in time, each step's nonlinear equation
solved by Newton's method with its exact Jacobian (the reference U^N of
Table 4).

algorithm3 (Algorithm 3): U_0^n = v; for l = 1, 2, ...: the linearised
system of eq. BDF-CQ-m-r-N,
    (dbar^alpha + A + g'(Ubar_{l-1})) W^n = fbar_n - (dbar^alpha + A) U_{l-1}^n - g(U_{l-1}^n),
with W^n = 0 for n <= 0 and Ubar_{l-1} the average of U_{l-1}^n over
n = 1..N, is solved by the WR iteration of eq. BDF-CQ-m-r-N-w from
W_{l,0} = 0, each sweep by Algorithm 1/2 (dense DFT in time, one sparse solve
per frequency with the spatial operator A + diag(g'(Ubar))), until
max |W_{l,m} - W_{l,m-1}| < the inner tolerance; then U_l = U_{l-1} + W_l.

Reading of the printed linearisation: eq. BDF-CQ-m-r-N prints the Jacobian
term as "- g'(Ubar) W"; the linearisation of + g(U) is + g'(Ubar) W, which is
what is implemented (the tests check that this reading reproduces Table 4).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bdf import corrected_source
from .cq import time_weights
from .sequential import _as_sparse
from .sweep import _phase


def g_cubic(u, c3, c1):
    return c3 * u ** 3 + c1 * u


def dg_cubic(u, c3, c1):
    return 3.0 * c3 * u ** 2 + c1


def nl_source(A, k, T, N, v, f, fder, c3, c1):
    """fbar_n, n = 1..N, of eq. BDF-CQ-m-r (the Table 1 correction carries g(v))."""
    A = _as_sparse(A)
    v = np.asarray(v, dtype=np.float64)
    M = A.shape[0]
    if f is None:
        f = np.zeros((N + 1, M))
    return corrected_source(k, T / N, f, A @ v + g_cubic(v, c3, c1), fder)


def nl_sequential(A, k, alpha, T, N, v, f, fder, c3, c1, newton_tol=1e-15, max_newton=50):
    """U^1..U^N of eq. BDF-CQ-m-r, every step solved by Newton's method."""
    A = _as_sparse(A)
    M = A.shape[0]
    tau = T / N
    ta = tau ** (-alpha)
    v = np.asarray(v, dtype=np.float64).reshape(M)
    w = time_weights(k, alpha, N + 1)
    fbar = nl_source(A, k, T, N, v, f, fder, c3, c1)
    D = np.zeros((N + 1, M))                  # D[n] = U^n - v
    U = np.zeros((N, M))
    I = sp.identity(M, format="csc")
    prev = v.copy()
    for n in range(1, N + 1):
        hist = ta * (w[1:n + 1][::-1] @ D[:n])    # tau^{-a} sum_{j=1..n} w_j (U^{n-j} - v)
        rhs = fbar[n - 1] - hist + ta * w[0] * v
        x = prev.copy()
        for _ in range(max_newton):
            F = ta * w[0] * x + A @ x + g_cubic(x, c3, c1) - rhs
            J = sp.csc_matrix(ta * w[0] * I + A + sp.diags(dg_cubic(x, c3, c1)))
            dx = spla.spsolve(J, -F)
            x = x + dx
            if np.max(np.abs(dx)) <= newton_tol * max(1.0, np.max(np.abs(x))):
                break
        U[n - 1] = x
        D[n] = x - v
        prev = x
    return U


class _Linearised:
    """The WR sweep of eq. BDF-CQ-m-r-N-w for one Newton step: the kappa-
    circulant all-at-once system of Algorithm 1/2 with zero history and the
    spatial operator A + diag(dg)."""

    def __init__(self, A, k, alpha, T, N, kappa, dg):
        self.A = _as_sparse(A)
        self.M = self.A.shape[0]
        self.N, self.kappa, self.alpha = N, kappa, alpha
        self.tau = T / N
        self.w = time_weights(k, alpha, N)
        self.Ad = sp.csc_matrix(self.A + sp.diags(dg))
        q = np.arange(N)
        self.scale = kappa ** (q / N)
        self.Vinv = _phase(N, -1) / N
        self.V = _phase(N, +1)
        j = np.arange(N)
        self.d = _phase(N, -1) @ (kappa ** (j / N) * self.w)

    def sweep(self, R, W_prev):
        """Direct form: P W_m = R + kappa tau^{-alpha} (Up (x) I) W_{m-1}."""
        N, ta = self.N, self.tau ** (-self.alpha)
        F = R.copy()
        for n in range(1, N + 1):
            for j in range(n, N):
                if self.w[j] != 0.0:
                    F[n - 1] += self.kappa * ta * self.w[j] * W_prev[N + n - j - 1]
        H = self.Vinv @ (self.scale[:, None] * F)
        Q = np.empty((N, self.M), dtype=np.complex128)
        tal = self.tau ** self.alpha
        I = sp.identity(self.M, dtype=np.complex128, format="csc")
        for p in range(N):
            Q[p] = spla.spsolve(sp.csc_matrix(self.d[p] * I + tal * self.Ad), tal * H[p])
        return ((self.V @ Q) / self.scale[:, None]).real


def newton_residual(A, k, alpha, T, N, v, fbar, U, c3, c1):
    """fbar_n - (dbar^alpha + A) U^n - g(U^n), n = 1..N (right side of eq. BDF-CQ-m-r-N)."""
    A = _as_sparse(A)
    tau = T / N
    ta = tau ** (-alpha)
    w = time_weights(k, alpha, N)
    D = U - v[None, :]
    R = np.empty_like(U)
    for n in range(1, N + 1):
        R[n - 1] = fbar[n - 1] - ta * (w[:n] @ D[n - 1::-1][:n]) - A @ U[n - 1] - g_cubic(U[n - 1], c3, c1)
    return R


def algorithm3(A, k, alpha, T, N, kappa, v, f, fder, c3, c1, newton_steps=3, inner_tol=1e-12, max_inner=50):
    """Algorithm 3.  Returns (iterates [U_0, U_1, ...], inner sweep counts per Newton step)."""
    A = _as_sparse(A)
    M = A.shape[0]
    v = np.asarray(v, dtype=np.float64).reshape(M)
    fbar = nl_source(A, k, T, N, v, f, fder, c3, c1)
    U = np.tile(v, (N, 1))
    its, counts = [U.copy()], []
    for _ in range(newton_steps):
        dg = dg_cubic(U.mean(axis=0), c3, c1)
        lin = _Linearised(A, k, alpha, T, N, kappa, dg)
        R = newton_residual(A, k, alpha, T, N, v, fbar, U, c3, c1)
        W = np.zeros((N, M))
        m = 0
        for m in range(1, max_inner + 1):
            Wn = lin.sweep(R, W)
            upd = np.max(np.abs(Wn - W))
            W = Wn
            if upd < inner_tol:
                break
        counts.append(m)
        U = U + W
        its.append(U.copy())
    return its, counts
