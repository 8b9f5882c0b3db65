"""Finite-difference Dirichlet Laplacian on a box (oracle; test infrastructure).

The paper's operator A is self-adjoint and coercive (Sec. 1, eqs. heat and
coe).  Here A = A_h is the standard (2d+1)-point finite-difference
discretisation of -Laplace on the box prod_i (0, len_i) with homogeneous
Dirichlet data and m_i interior points per direction, h_i = len_i/(m_i+1).
Unknowns are ordered with x fastest, then y, then z.
"""
import numpy as np
import scipy.sparse as sp


class Grid:
    def __init__(self, m, length=None):
        self.m = tuple(int(x) for x in m)
        self.dim = len(self.m)
        if not 1 <= self.dim <= 3:
            raise ValueError("dim must be 1, 2 or 3")
        self.length = tuple(float(x) for x in (length or [1.0] * self.dim))
        self.h = tuple(L / (mi + 1) for L, mi in zip(self.length, self.m))
        self.M = int(np.prod(self.m))

    def coords(self, axis):
        """Interior node coordinates along one axis."""
        return self.h[axis] * np.arange(1, self.m[axis] + 1)


def _second_difference(m, h):
    e = np.ones(m)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr") / h ** 2


def laplacian(grid):
    """Sparse A_h (M x M), x fastest."""
    ops = [_second_difference(mi, hi) for mi, hi in zip(grid.m, grid.h)]
    eye = [sp.identity(mi, format="csr") for mi in grid.m]
    A = sp.csr_matrix((grid.M, grid.M))
    for axis in range(grid.dim):
        # Kronecker order: slowest axis first (z, y, x).
        factors = []
        for a in reversed(range(grid.dim)):
            factors.append(ops[a] if a == axis else eye[a])
        term = factors[0]
        for F in factors[1:]:
            term = sp.kron(term, F, format="csr")
        A = A + term
    return A.tocsr()


def sine_eigenvalues(m, h):
    """Eigenvalues (4/h^2) sin^2(j pi / (2(m+1))), j = 1..m, of one
    second-difference factor; the matching eigenvector is sin(j pi x / len)."""
    j = np.arange(1, m + 1)
    return (4.0 / h ** 2) * np.sin(j * np.pi / (2.0 * (m + 1))) ** 2


def l2h(grid, u):
    """Discrete L2(Omega) norm (h^d sum u^2)^{1/2}, the norm of e_m^N (Sec. 4)."""
    return float(np.sqrt(np.prod(grid.h) * np.sum(np.asarray(u) ** 2)))
