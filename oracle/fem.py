"""P1 finite elements in 1D: the paper's own spatial discretisation (oracle;
test infrastructure).

Sec. 4 (opening of the numerical experiments) discretises space by the
Galerkin method with continuous piecewise-linear elements on a uniform mesh
of (0, 1): the semi-discrete problem is M_h d_t^alpha u_h + K_h u_h = F_h
with the mass matrix M_h = (phi_j, phi_i) = h/6 tridiag(1, 4, 1), the
stiffness matrix K_h = (phi_j', phi_i') = (1/h) tridiag(-1, 2, -1) and the
load F_h(t)_i = (f(t), phi_i).  Divided by h this reads

    Mt d_t^alpha u + A u = Ft,   Mt = tridiag(1, 4, 1)/6,  A = K_h/h,  Ft = F_h/h,

where A is exactly the finite-difference A_h of ``oracle.grid``.  The time
schemes are those of Sec. 2.1 / 3.1 with the mass matrix on the time
derivative (the corrected source keeps its form: Ftbar_n = Ft(t_n) +
a_n (Ft(0) - A v) + sum_l b_{l,n} tau^l d^l Ft/dt^l (0), Table 1).  One WR
sweep is the kappa-circulant all-at-once system
    tau^{-alpha} (B_k(kappa) (x) Mt) U_m + (I (x) A) U_m = F_{m-1},
diagonalised in time exactly as in Algorithms 1 and 2; Step 2 becomes
(d_p Mt + tau^alpha A) Q_p = tau^alpha H_p.

The data of a FEM problem are the nodal values of v_h (for the paper's
examples its L2 projection, M_h^{-1} (v, phi_i)) and the scaled loads Ft,
d^l Ft/dt^l (0) at the nodes.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .cq import time_weights
from .grid import Grid, laplacian
from .sequential import refined_solver, source_terms
from .sweep import Problem


def mass_scaled(m):
    """Mt = M_h / h = tridiag(1, 4, 1)/6 on m interior nodes (sparse CSR)."""
    e = np.ones(m)
    return sp.diags([e[:-1], 4.0 * e, e[:-1]], [-1, 0, 1], format="csr") / 6.0


def stiffness_scaled(m, length=1.0):
    """A = K_h / h = (1/h^2) tridiag(-1, 2, -1), the FD A_h of the same mesh."""
    return laplacian(Grid((m,), (length,)))


def l2_fe(m, u, length=1.0):
    """L2(0, len) norm of the P1 function with nodal values u: (u^T M_h u)^{1/2}."""
    h = length / (m + 1)
    u = np.asarray(u, dtype=np.float64)
    return float(np.sqrt(h * (u @ (mass_scaled(m) @ u))))


def fem_sequential(m, k, alpha, T, N, v, F=None, Fder=None, length=1.0):
    """O1 with the mass matrix: U^1..U^N of
        Mt tau^{-alpha} sum_{j=0..n} omega_j (U^{n-j} - v) + A U^n = Ftbar_n,
    each step solving (omega_0 Mt + tau^alpha A) U^n
        = Mt (sum_{j=1..n} omega_j (v - U^{n-j}) + omega_0 v) + tau^alpha Ftbar_n
    (LU plus long-double iterative refinement, as in ``oracle.sequential``)."""
    Mt = mass_scaled(m)
    A = stiffness_scaled(m, length)
    tau = T / N
    v = np.asarray(v, dtype=np.float64).reshape(m)
    w = time_weights(k, alpha, N + 1)
    fbar = source_terms(A, k, alpha, T, N, v, F, Fder)
    lu = spla.splu(sp.csc_matrix(w[0] * Mt + tau ** alpha * A))
    solve = refined_solver(lu, w[0], tau ** alpha, A, mass=Mt)
    D = np.zeros((N + 1, m))          # D[n] = U^n - v
    U = np.zeros((N, m))
    for n in range(1, N + 1):
        hist = -(w[1:n + 1][::-1] @ D[:n])
        U[n - 1] = solve(Mt @ (hist + w[0] * v) + tau ** alpha * fbar[n - 1])
        D[n] = U[n - 1] - v
    return U


class FemProblem(Problem):
    """O2 with the mass matrix: the sweep of Algorithm 1/2 on the FEM system.
    Same interface as ``oracle.sweep.Problem`` (sweep, solve_P, direct and
    residual forms); the mass matrix multiplies the time-derivative terms."""

    def __init__(self, m, k, alpha, T, N, kappa, v, F=None, Fder=None, length=1.0):
        super().__init__(stiffness_scaled(m, length), k, alpha, T, N, kappa, v, F, Fder)
        self.Mt = mass_scaled(m)
        ta = self.tau ** (-self.alpha)
        # G_n = Ftbar_n + tau^{-alpha} s_n Mt v
        self.G = self.fbar + ta * np.outer(self.s, self.Mt @ self.v)

    def direct_rhs(self, U_prev):
        N, ta = self.N, self.tau ** (-self.alpha)
        F = self.G.copy()
        for n in range(1, N + 1):
            acc = np.zeros(self.M)
            for j in range(n, N):
                if self.w[j] != 0.0:
                    acc += self.w[j] * U_prev[N + n - j - 1]
            F[n - 1] += self.kappa * ta * (self.Mt @ acc)
        return F

    def apply_T(self, U):
        """(T U)_n = tau^{-alpha} Mt sum_{j=0..n-1} omega_j U^{n-j} + A U^n."""
        N, ta = self.N, self.tau ** (-self.alpha)
        out = np.zeros_like(U)
        for n in range(1, N + 1):
            out[n - 1] = ta * (self.Mt @ (self.w[:n] @ U[n - 1::-1][:n])) + self.A @ U[n - 1]
        return out

    def shifted_solve(self, p, b, refine=2):
        """(d_p Mt + tau^alpha A) x = b: sparse LU plus iterative refinement with
        the residual in long double (as in ``Problem.shifted_solve``)."""
        ta = self.tau ** self.alpha
        Mt_c = sp.csc_matrix(self.Mt, dtype=np.complex128)
        lu = spla.splu(sp.csc_matrix(self.d[p] * Mt_c + ta * sp.csc_matrix(self.A, dtype=np.complex128)))
        x = lu.solve(b)
        if refine:
            A_ld = sp.csr_matrix(self.A, dtype=np.longdouble)
            Mt_ld = sp.csr_matrix(self.Mt, dtype=np.longdouble)
            d_ld = np.clongdouble(self.d[p])
            ta_ld = np.longdouble(self.tau) ** np.longdouble(self.alpha)
            b_ld = b.astype(np.clongdouble)
            for _ in range(refine):
                x_ld = x.astype(np.clongdouble)
                r = b_ld - (d_ld * (Mt_ld @ x_ld) + ta_ld * (A_ld @ x_ld))
                x = x + lu.solve(r.astype(np.complex128))
        return x
