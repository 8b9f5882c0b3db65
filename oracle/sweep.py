"""O2: one waveform-relaxation sweep solved by diagonalization in time, with
dense DFT matrices (oracle; test infrastructure).

All-at-once system of one sweep (Sec. 2.2 eqs. BDF-k-matrix and BDF-k-F;
Sec. 3.2 eqs. BDF-k-matrix-frac and BDF-subdiff-F):
    tau^{-alpha} (B_k(kappa) (x) I) U_m + (I (x) A) U_m = F_{m-1},
    B[n, j] = omega_{n-j}             (n >= j)
            = kappa omega_{N+n-j}     (n <  j)     (1-based n, j = 1..N),
    F_n = fbar_n + tau^{-alpha} s_n v + kappa tau^{-alpha} sum_{j=n..N-1} omega_j U_{m-1}^{N+n-j},
    s_n = sum_{j=0..n-1} omega_j.
For BDF-k the weights vanish beyond k, so only rows n <= k carry the
kappa term (this is the reading of eq. BDF-k-F that agrees with eq. BDF-iter
and with the matrix B_k(kappa); the printed upper index of that sum is a typo).

Diagonalization (Lemmas diag-heat and diag-frac): B = S D S^{-1}, S = Lambda V,
Lambda = diag(kappa^{-q/N}), V[q, p] = exp(+2 pi i p q / N), q, p = 0..N-1, and
D = diag(d_p) with d_p the eigenvalues of the circulant whose first column is
kappa^{j/N} omega_j, i.e. d_p = sum_j kappa^{j/N} omega_j exp(-2 pi i j p / N).

Algorithm 1 / 2:
    Step 1  H = S^{-1} F                    (scale row q by kappa^{q/N}, then V^{-1} = V^H / N)
    Step 2  (d_p I + tau^alpha A) Q_p = tau^alpha H_p       for every p = 0..N-1
    Step 3  U = S Q                         (V, then scale row q by kappa^{-q/N})

Two forms of the sweep are provided; they are the same iteration in exact
arithmetic because P - T = kappa tau^{-alpha} (Up (x) I):
    direct    U_m = P^{-1} F_{m-1}                    (the paper's literal form)
    residual  U_m = U_{m-1} + P^{-1} (G - T U_{m-1}),
              G_n = fbar_n + tau^{-alpha} s_n v,
              (T U)_n = tau^{-alpha} sum_{j=0..n-1} omega_j U^{n-j} + A U^n.
All N frequencies are solved (no use of Hermitian symmetry), and the
imaginary part of the result is returned so that its smallness can be checked.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cq import time_weights
from .sequential import _as_sparse, source_terms


def _phase(N, sign):
    """Dense matrix exp(sign 2 pi i p q / N); p q is reduced mod N before scaling
    (exact, by periodicity) so the phase is accurate for large N."""
    q = np.arange(N)
    return np.exp(sign * 2j * np.pi * (np.outer(q, q) % N) / N)


def eigenvalues(k, alpha, N, kappa):
    """d_p, p = 0..N-1: eigenvalues of the scaled circulant (dense DFT of its first column)."""
    w = time_weights(k, alpha, N)
    j = np.arange(N)
    c = kappa ** (j / N) * w
    return _phase(N, -1) @ c


class Problem:
    """Everything one sweep needs that does not depend on the iterate."""

    def __init__(self, A, k, alpha, T, N, kappa, v, f=None, fder=None):
        self.A = _as_sparse(A)
        self.M = self.A.shape[0]
        self.k, self.alpha, self.T, self.N, self.kappa = k, float(alpha), float(T), int(N), float(kappa)
        self.tau = self.T / self.N
        self.v = np.asarray(v, dtype=np.float64).reshape(self.M)
        self.w = time_weights(k, self.alpha, N)
        s = np.concatenate([[0.0], np.cumsum(self.w)])[:N + 1]      # s[n] = sum_{j<n} omega_j
        self.s = s[1:]                                              # s_n, n = 1..N
        self.fbar = source_terms(self.A, k, self.alpha, self.T, N, self.v, f, fder)
        ta = self.tau ** (-self.alpha)
        self.G = self.fbar + ta * np.outer(self.s, self.v)
        q = np.arange(N)
        self.scale = kappa ** (q / N)                               # Lambda^{-1} diagonal
        self.Vinv = _phase(N, -1) / N
        self.V = _phase(N, +1)
        self.d = eigenvalues(k, self.alpha, N, kappa)

    # -- the kappa-circulant operator and its pieces ------------------------
    def direct_rhs(self, U_prev):
        """F_{m-1} of eq. BDF-k-F / BDF-subdiff-F."""
        N, ta = self.N, self.tau ** (-self.alpha)
        F = self.G.copy()
        for n in range(1, N + 1):
            for j in range(n, N):
                if self.w[j] != 0.0:
                    F[n - 1] += self.kappa * ta * self.w[j] * U_prev[N + n - j - 1]
        return F

    def apply_T(self, U):
        """(T U)_n = tau^{-alpha} sum_{j=0..n-1} omega_j U^{n-j} + A U^n."""
        N, ta = self.N, self.tau ** (-self.alpha)
        out = np.zeros_like(U)
        for n in range(1, N + 1):
            out[n - 1] = ta * (self.w[:n] @ U[n - 1::-1][:n]) + self.A @ U[n - 1]
        return out

    def shifted_solve(self, p, b, refine=2):
        """Step 2 for frequency p: the solution of (d_p I + tau^alpha A) x = b.

        A sparse LU solve, followed by `refine` steps of iterative refinement
        whose residual is formed in extended precision (long double), so that x
        is the exact solution rounded to FP64 rather than carrying the
        factorisation's error of order eps times the condition number of the
        shifted Laplacian (which grows like (m+1)^2)."""
        M, ta = self.M, self.tau ** self.alpha
        I = sp.identity(M, dtype=np.complex128, format="csc")
        lu = spla.splu(sp.csc_matrix(self.d[p] * I + ta * sp.csc_matrix(self.A, dtype=np.complex128)))
        x = lu.solve(b)
        if refine:
            A_ld = sp.csr_matrix(self.A, dtype=np.longdouble)
            d_ld = np.clongdouble(self.d[p])
            ta_ld = np.longdouble(self.tau) ** np.longdouble(self.alpha)
            b_ld = b.astype(np.clongdouble)
            for _ in range(refine):
                x_ld = x.astype(np.clongdouble)
                r = b_ld - (d_ld * x_ld + ta_ld * (A_ld @ x_ld))
                x = x + lu.solve(r.astype(np.complex128))
        return x

    def solve_P(self, X, refine=2):
        """P^{-1} X by Algorithm 1/2 (dense DFT, all N frequencies).
        Returns (real part, max abs imaginary part)."""
        N, M, ta = self.N, self.M, self.tau ** self.alpha
        H = self.Vinv @ (self.scale[:, None] * X)                  # Step 1
        Q = np.empty((N, M), dtype=np.complex128)
        for p in range(N):                                          # Step 2
            Q[p] = self.shifted_solve(p, ta * H[p], refine)
        Y = (self.V @ Q) / self.scale[:, None]                      # Step 3
        return Y.real.copy(), float(np.max(np.abs(Y.imag))) if Y.size else 0.0

    def sweep(self, U_prev, form="direct"):
        """One WR sweep; returns (U_m, max abs imaginary part of the raw result)."""
        U_prev = np.asarray(U_prev, dtype=np.float64).reshape(self.N, self.M)
        if form == "direct":
            return self.solve_P(self.direct_rhs(U_prev))
        if form == "residual":
            delta, im = self.solve_P(self.G - self.apply_T(U_prev))
            return U_prev + delta, im
        raise ValueError("form must be 'direct' or 'residual'")


def initial_iterate(prob, init="v"):
    """U_0: v at every level (Thm 2.6 / Thm 3.5) or zero (reproduces Tables 2-3)."""
    if init == "v":
        return np.tile(prob.v, (prob.N, 1))
    if init == "zero":
        return np.zeros((prob.N, prob.M))
    raise ValueError(init)


def iterate(prob, sweeps, init="v", form="direct", U0=None):
    """Run `sweeps` sweeps; returns the list [U_0, U_1, ..., U_sweeps]."""
    U = initial_iterate(prob, init) if U0 is None else np.array(U0, dtype=np.float64)
    out = [U]
    for _ in range(sweeps):
        U, _ = prob.sweep(U, form)
        out.append(U)
    return out
