"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the
CPU oracle.

This module holds none of the method's arithmetic: it only draws seeded
random sine-mode coefficients and evaluates the resulting initial values v,
sources f(t_n) and time derivatives d^l f/dt^l (0) on the interior grid
nodes.  Everything is FP64 NumPy on the host.

Workloads (all on boxes with homogeneous Dirichlet data, len = 1):

* ``heat1d``   1D, m = 63, N = 64, BDF2, T = 1, kappa = 1e-3;
               v = sin(pi x) + sum_{j<=8} (z_j / j^2) sin(j pi x),
               f = sum_{j<=4} b_j sin(j pi x) cos(2 pi j t).
* ``heat2d``   2D, 255 x 255, N = 512, BDF4, T = 1, kappa = 1e-5;
               v, f(., 0) = sum_{i,j<=16} z_ij/(i^2+j^2) sin(i pi x) sin(j pi y)
               (independent draws), f(x, t) = f(x, 0) cos(2 pi t).
* ``subdiff2d`` 2D, 511 x 511, N = 1024, CQ-BDF3, alpha = 0.5, T = 1,
               kappa = 1e-4; v = 1 on [0.25, 0.75]^2 (closed) plus 1e-3 z per
               node, f = 0.
* ``heat3d``   3D, 127^3, N = 256, BDF6, T = 1, kappa = 1e-6; as heat2d with
               8 x 8 x 8 modes decaying as 1/(i^2+j^2+l^2).
* ``batch``    instance i of a many-instance batch, seed (4, i): dim 1 or 2,
               m per dim uniform in 63..1023, N a power of two in 32..1024,
               k uniform in 1..6, alpha in {1, 0.3, 0.7},
               kappa = 10^U(-6, -2); data as heat1d / heat2d.
* ``example1`` Sec. 4 Example 1: 1D, h = 1/1000, T = 0.5, N = 100,
               kappa = 0.5, v = indicator of (0, 1/2), f = e^t cos x.
* ``example2`` Sec. 4 Example 2: 1D, h = 1/1000, alpha = 0.5, T = 0.1,
               N = 100, kappa = 0.1, v = discrete Dirac at x = 1/2
               (value 1/h at that node), f = 0.
* ``example4`` Sec. 4 Example 4 (semilinear, Allen-Cahn term): 1D,
               h = 1/1000, T = 0.4, N = 100, kappa = 0.1, v = 0, f from the
               manufactured solution t^2/2 sin(2 pi x).

Sizes can be shrunk (``m``, ``N`` keywords) for parity tests at sizes the
oracle finishes in seconds; the recipe stays the same.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    m: tuple                 # interior points per dimension
    k: int
    alpha: float
    T: float
    N: int
    kappa: float
    v: np.ndarray            # [M]
    f: Optional[np.ndarray]  # [N+1, M] or None (f = 0)
    fder: Optional[np.ndarray]  # [k-2, M] or None
    tol: float = 1e-12
    length: tuple = field(default=None)
    # sine-series coefficients of the data when it is a finite sine series:
    # {"v": c_v, "f": c_f} with c[i, j, ...] the coefficient of
    # sin((i+1) pi x) sin((j+1) pi y) ...; f(x, t) = cos(2 pi t) * series(c_f)
    modes: Optional[dict] = None
    # spatial discretisation: "fd" (finite differences; f holds the source) or
    # "fem" (1D P1 elements; f holds the scaled loads (f(t), phi_i)/h)
    space: str = "fd"

    @property
    def dim(self):
        return len(self.m)

    @property
    def M(self):
        return int(np.prod(self.m))


def _nodes(m):
    return np.arange(1, m + 1) / (m + 1.0)


def _sine_field(m, coeffs):
    """sum over modes c[i, j, ...] prod_axis sin((idx+1) pi x_axis), x fastest."""
    dim = len(m)
    out = np.zeros(tuple(reversed(m)))
    basis = [np.sin(np.pi * np.outer(np.arange(1, coeffs.shape[a] + 1), _nodes(m[a])))
             for a in range(dim)]
    if dim == 1:
        out = coeffs @ basis[0]
    elif dim == 2:
        # out[y, x] = sum_ij c[i, j] sin(i pi x) sin(j pi y)
        out = basis[1].T @ coeffs.T @ basis[0]
    else:
        # out[z, y, x] = sum_ijl c[i, j, l] sin(i pi x) sin(j pi y) sin(l pi z)
        out = np.einsum("ijl,ix,jy,lz->zyx", coeffs, basis[0], basis[1], basis[2], optimize=True)
    return np.ascontiguousarray(out).reshape(-1)


def _decay(shape):
    idx = np.meshgrid(*[np.arange(1, s + 1) for s in shape], indexing="ij")
    return 1.0 / sum(i.astype(np.float64) ** 2 for i in idx)


def _cos_profile_derivs(N, T, k, spatial):
    """f(t_n) = spatial cos(2 pi t_n) and d^l/dt^l at 0 for l = 1..k-2."""
    t = T * np.arange(N + 1) / N
    f = np.cos(2 * np.pi * t)[:, None] * spatial[None, :]
    fder = None
    if k > 2:
        rows = []
        for l in range(1, k - 1):
            # d^l/dt^l cos(2 pi t) at t = 0: (2 pi)^l cos(l pi / 2)
            c = (2 * np.pi) ** l * [1.0, 0.0, -1.0, 0.0][l % 4]
            rows.append(c * spatial)
        fder = np.array(rows)
    return f, fder


def heat1d(seed=1, m=63, N=64, k=2, T=1.0, kappa=1e-3, tol=1e-12):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(8)
    b = rng.standard_normal(4)
    x = _nodes(m)
    v = np.sin(np.pi * x) + sum(z[j - 1] / j ** 2 * np.sin(j * np.pi * x) for j in range(1, 9))
    t = T * np.arange(N + 1) / N
    f = sum(b[j - 1] * np.outer(np.cos(2 * np.pi * j * t), np.sin(j * np.pi * x)) for j in range(1, 5))
    fder = None
    if k > 2:
        rows = []
        for l in range(1, k - 1):
            rows.append(sum(b[j - 1] * (2 * np.pi * j) ** l * [1.0, 0.0, -1.0, 0.0][l % 4]
                            * np.sin(j * np.pi * x) for j in range(1, 5)))
        fder = np.array(rows)
    return Workload("heat1d", (m,), k, 1.0, T, N, kappa, v, f, fder, tol)


def heat2d(seed=2, m=(255, 255), N=512, k=4, T=1.0, kappa=1e-5, modes=16, tol=1e-12):
    m = tuple(m)
    rng = np.random.default_rng(seed)
    nm = (min(modes, m[0]), min(modes, m[1]))
    cv = rng.standard_normal(nm) * _decay(nm)
    cf = rng.standard_normal(nm) * _decay(nm)
    v = _sine_field(m, cv)
    f, fder = _cos_profile_derivs(N, T, k, _sine_field(m, cf))
    return Workload("heat2d", m, k, 1.0, T, N, kappa, v, f, fder, tol, modes={"v": cv, "f": cf})


def subdiff2d(seed=3, m=(511, 511), N=1024, k=3, alpha=0.5, T=1.0, kappa=1e-4, tol=1e-12):
    m = tuple(m)
    rng = np.random.default_rng(seed)
    xs = [_nodes(mi) for mi in m]
    inside = [((x >= 0.25) & (x <= 0.75)).astype(np.float64) for x in xs]
    v = np.outer(inside[1], inside[0]).reshape(-1) + 1e-3 * rng.standard_normal(int(np.prod(m)))
    return Workload("subdiff2d", m, k, alpha, T, N, kappa, v, None, None, tol)


def heat3d(seed=5, m=(127, 127, 127), N=256, k=6, T=1.0, kappa=1e-6, modes=8, tol=1e-12):
    m = tuple(m)
    rng = np.random.default_rng(seed)
    nm = tuple(min(modes, mi) for mi in m)
    cv = rng.standard_normal(nm) * _decay(nm)
    cf = rng.standard_normal(nm) * _decay(nm)
    v = _sine_field(m, cv)
    f, fder = _cos_profile_derivs(N, T, k, _sine_field(m, cf))
    return Workload("heat3d", m, k, 1.0, T, N, kappa, v, f, fder, tol, modes={"v": cv, "f": cf})


def batch_params(i, seed=4, m_range=(63, 1023), N_choices=(32, 64, 128, 256, 512, 1024)):
    """(dim, m, N, k, alpha, kappa, data seed) of instance i of the many-instance batch."""
    rng = np.random.default_rng([seed, i])
    dim = int(rng.integers(1, 3))
    m = tuple(int(rng.integers(m_range[0], m_range[1] + 1)) for _ in range(dim))
    N = int(rng.choice(N_choices))
    k = int(rng.integers(1, 7))
    alpha = float(rng.choice([1.0, 0.3, 0.7]))
    kappa = float(10.0 ** rng.uniform(-6, -2))
    dseed = int(rng.integers(0, 2 ** 31))
    return dim, m, N, k, alpha, kappa, dseed


def batch_instance(i, seed=4, m_range=(63, 1023), N_choices=(32, 64, 128, 256, 512, 1024)):
    """Instance i of the many-instance batch (parameters and data)."""
    dim, m, N, k, alpha, kappa, dseed = batch_params(i, seed, m_range, N_choices)
    if dim == 1:
        w = heat1d(seed=dseed, m=m[0], N=N, k=k, kappa=kappa)
    else:
        w = heat2d(seed=dseed, m=m, N=N, k=k, kappa=kappa)
    w.name, w.alpha = "batch", alpha
    return w


def example1(k, M=999, N=100):
    """Sec. 4, Example 1 (Table 2)."""
    x = _nodes(M)
    T = 0.5
    v = (x < 0.5).astype(np.float64)
    t = T * np.arange(N + 1) / N
    f = np.exp(t)[:, None] * np.cos(x)[None, :]
    fder = np.tile(np.cos(x), (k - 2, 1)) if k > 2 else None
    return Workload("example1", (M,), k, 1.0, T, N, 0.5, v, f, fder, 1e-12)


def example2(k, M=999, N=100):
    """Sec. 4, Example 2 (Table 3)."""
    v = np.zeros(M)
    v[(M + 1) // 2 - 1] = M + 1.0          # node x = 1/2, value 1/h
    return Workload("example2", (M,), k, 0.5, 0.1, N, 0.1, v, None, None, 1e-12)


def example4(k, alpha, M=999, N=100, eps=1.0):
    """Sec. 4, Example 4 (Table 4): 1D Allen-Cahn term g(u) = (u^3 - u)/eps^2,
    T = 0.4, kappa = 0.1, v = 0, f such that u = t^2/Gamma(3) sin(2 pi x) solves
    the continuous problem: f = t^{2-alpha}/Gamma(3-alpha) sin(2 pi x)
    + (2 pi)^2 u + g(u).  Returns (workload, c3, c1); d^l f/dt^l (0) = 0."""
    from math import gamma
    T = 0.4
    x = _nodes(M)
    t = T * np.arange(N + 1) / N
    s = np.sin(2 * np.pi * x)
    u = (t ** 2 / gamma(3.0))[:, None] * s[None, :]
    f = (t ** (2 - alpha) / gamma(3.0 - alpha))[:, None] * s[None, :] + (2 * np.pi) ** 2 * u + (u ** 3 - u) / eps ** 2
    fder = np.zeros((k - 2, M)) if k > 2 else None
    w = Workload("example4", (M,), k, alpha, T, N, 0.1, np.zeros(M), f, fder, 1e-12)
    return w, 1.0 / eps ** 2, -1.0 / eps ** 2


def _hat_integral(x, h, a, b):
    """Integral over (a, b) of the hat function of node x (support x - h .. x + h)."""
    def prim(s):   # antiderivative of the hat from x - h, s clipped to the support
        s = min(max(s, x - h), x + h)
        if s <= x:
            return (s - x + h) ** 2 / (2 * h)
        return h / 2 + (s - x) - (s - x) ** 2 / (2 * h)
    return prim(b) - prim(a) if b > a else 0.0


def _l2_projection(load_over_h):
    """Nodal values of the P1 L2 projection from the scaled load (v, phi_i)/h:
    the solve of tridiag(1, 4, 1)/6 y = load/h (Dirichlet nodes excluded)."""
    from scipy.linalg import solve_banded
    m = load_over_h.shape[0]
    ab = np.zeros((3, m))
    ab[0, 1:] = 1.0 / 6.0
    ab[1, :] = 4.0 / 6.0
    ab[2, :-1] = 1.0 / 6.0
    return solve_banded((1, 1), ab, load_over_h)


def example1_fem(k, M=999, N=100):
    """Sec. 4, Example 1 (Table 2) with the paper's P1 elements: v_h the L2
    projection of the indicator of (0, 1/2); Ft(t)_i = (e^t cos x, phi_i)/h
    = e^t cos(x_i) 2 (1 - cos h)/h^2 exactly; its time derivatives likewise."""
    h = 1.0 / (M + 1)
    x = _nodes(M)
    T = 0.5
    load_v = np.array([_hat_integral(xi, h, 0.0, 0.5) for xi in x]) / h
    v = _l2_projection(load_v)
    t = T * np.arange(N + 1) / N
    g = np.cos(x) * 2.0 * (1.0 - np.cos(h)) / h ** 2
    f = np.exp(t)[:, None] * g[None, :]
    fder = np.tile(g, (k - 2, 1)) if k > 2 else None
    w = Workload("example1_fem", (M,), k, 1.0, T, N, 0.5, v, f, fder, 1e-12)
    w.space = "fem"
    return w


def example2_fem(k, M=999, N=100):
    """Sec. 4, Example 2 (Table 3) with P1 elements: v_h the L2 projection of
    delta_{1/2}, whose load (delta, phi_i) = phi_i(1/2); f = 0."""
    h = 1.0 / (M + 1)
    x = _nodes(M)
    load_v = np.maximum(0.0, 1.0 - np.abs(x - 0.5) / h) / h
    v = _l2_projection(load_v)
    w = Workload("example2_fem", (M,), k, 0.5, 0.1, N, 0.1, v, None, None, 1e-12)
    w.space = "fem"
    return w


def fem1d(seed=61, m=63, N=64, k=2, alpha=1.0, T=1.0, kappa=1e-3, tol=1e-12):
    """A 1D P1 problem with smooth random data: v_h nodal values of 8 sine modes
    with N(0,1)/j^2 amplitudes, scaled loads Ft = 4 sine modes x cos(2 pi j t)."""
    w = heat1d(seed=seed, m=m, N=N, k=k, T=T, kappa=kappa, tol=tol)
    w.name, w.alpha, w.space = "fem1d", alpha, "fem"
    return w


CONFIGS = {
    "heat1d": heat1d,
    "heat2d": heat2d,
    "subdiff2d": subdiff2d,
    "heat3d": heat3d,
}
