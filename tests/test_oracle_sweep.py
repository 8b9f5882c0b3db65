"""Pins of the oracle's sequential stepper (O1), diagonalized sweep (O2) and
dense all-at-once solve (O3) against the paper's printed worked examples,
closed forms, brute force and invariants."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.bruteforce import all_at_once, kappa_circulant, lower_toeplitz
from oracle.contraction import spectral_radius
from oracle.cq import time_weights
from oracle.grid import Grid, l2h, laplacian, sine_eigenvalues
from oracle.sequential import sequential, source_terms
from oracle.sweep import Problem, iterate
from paper_2007_13125_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([float(x) for x in line.split()[1:]])
    return np.array(rows)


def _printed_match(got, printed):
    """got agrees with a 3-significant-digit printed value to within one unit in
    the last printed digit (plus the rounding half-unit)."""
    e = np.floor(np.log10(abs(printed)))
    unit = 10.0 ** (e - 2)
    return abs(got - printed) <= 1.5 * unit


def _table_errors(w, sweeps=3):
    g = Grid(w.m)
    A = laplacian(g)
    U = sequential(A, w.k, w.alpha, w.T, w.N, w.v, w.f, w.fder)
    prob = Problem(A, w.k, w.alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    its = iterate(prob, sweeps, init="zero", form="direct")
    return [l2h(g, Ui[-1] - U[-1]) for Ui in its]


@pytest.mark.parametrize("k", range(1, 7))
def test_table2_example1(k):
    # PIN-4: Sec. 4 Example 1, Table 2, rows m = 0..3 (rows 4-5 are at the roundoff floor).
    printed = _golden("table2.txt")[:, k - 1]
    got = _table_errors(wl.example1(k))
    for m in range(4):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])


@pytest.mark.parametrize("k", range(1, 7))
def test_table3_example2(k):
    # PIN-4: Sec. 4 Example 2, Table 3, rows m = 0..3.  The paper's runs use P1 finite
    # elements; the FD Laplacian agrees to within one unit in the last printed digit.
    printed = _golden("table3.txt")[:, k - 1]
    got = _table_errors(wl.example2(k))
    for m in range(4):
        assert _printed_match(got[m], printed[m]), (k, m, got[m], printed[m])


def test_printed_index_of_F_diverges():
    # Reading of eq. BDF-k-F: its printed relaxation sum, sum_{j=1..n} omega_j U_{m-1}^{N-j+1},
    # disagrees with eq. BDF-iter and with B_k(kappa).  Used literally, the sweep does not
    # reproduce Table 2 (it diverges), so the oracle takes sum_{j=n..k} omega_j U^{N+n-j}.
    w = wl.example1(2)
    g = Grid(w.m)
    A = laplacian(g)

    class Printed(Problem):
        def direct_rhs(self, U_prev):
            F = self.G.copy()
            for n in range(1, self.N + 1):
                for j in range(1, min(n, self.k) + 1):
                    F[n - 1] += self.kappa / self.tau * self.w[j] * U_prev[self.N - j]
            return F

    U = sequential(A, w.k, 1.0, w.T, w.N, w.v, w.f, w.fder)
    prob = Printed(A, w.k, 1.0, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    its = iterate(prob, 3, init="zero", form="direct")
    errs = [l2h(g, Ui[-1] - U[-1]) for Ui in its]
    printed = _golden("table2.txt")[:, 1]
    # sweep 1 starts from U_0 = 0, so the coupling first shows in sweep 2
    assert not _printed_match(errs[2], printed[2])
    assert errs[3] > errs[2]


def test_contraction_bdf1_closed_form():
    # PIN-5: BDF1 factor kappa R^N / (1 - kappa R^N), R = 1/(1 + tau mu) (Remark 2.3).
    for T, N, kappa, mu in [(0.5, 100, 0.5, np.pi ** 2), (1.0, 64, 0.1, 3.0), (0.2, 40, 0.3, 50.0)]:
        tau = T / N
        R = 1.0 / (1.0 + tau * mu)
        ref = kappa * R ** N / (1.0 - kappa * R ** N)
        assert abs(spectral_radius(1, 1.0, T, N, kappa, mu) - ref) <= 1e-6 * ref


@pytest.mark.parametrize("k", range(2, 7))
def test_contraction_matches_table2_ratio(k):
    # The slowest mode of Example 1 is sin(pi x) (mu ~ pi^2); its factor is the ratio of
    # successive rows of Table 2 (to the 3 printed digits).
    h = 1.0 / 1000
    mu = sine_eigenvalues(999, h)[0]
    rho = spectral_radius(k, 1.0, 0.5, 100, 0.5, mu)
    t2 = _golden("table2.txt")[:, k - 1]
    assert abs(rho - t2[2] / t2[1]) <= 0.01 * rho
    assert abs(rho - t2[3] / t2[2]) <= 0.01 * rho


@pytest.mark.parametrize("k,alpha", [(1, 1.0), (3, 1.0), (6, 1.0), (2, 0.5), (4, 0.3)])
def test_sweep_error_ratio_equals_spectral_radius(k, alpha):
    # One eigenmode, many sweeps: the observed error ratio of O2 approaches rho(J).
    T, N, kappa, mu = 1.0, 32, 0.5, 0.5
    v = np.array([1.0])
    U = sequential(np.array([[mu]]), k, alpha, T, N, v)
    prob = Problem(np.array([[mu]]), k, alpha, T, N, kappa, v)
    its = iterate(prob, 5, init="zero", form="residual")
    err = [np.max(np.abs(Ui - U)) for Ui in its]
    rho = spectral_radius(k, alpha, T, N, kappa, mu)
    assert rho > 1e-3
    assert abs(err[4] / err[3] - rho) <= 0.05 * rho


def test_smaller_kappa_contracts_faster_and_ratio_independent_of_N():
    # PIN-13: Sec. 4 Example 1 discussion and Remark 2.3.
    mu = np.pi ** 2
    rhos = [spectral_radius(3, 1.0, 0.5, 200, kap, mu) for kap in (0.5, 0.1, 0.01)]
    assert rhos[0] > rhos[1] > rhos[2]
    byN = [spectral_radius(3, 1.0, 0.5, N, 0.1, mu) for N in (50, 100, 200, 400)]
    assert max(byN) / min(byN) < 1.1


@pytest.mark.parametrize("m,length", [(1, 1.0), (7, 1.0), (100, 1.0), (255, 2.0), (999, 0.5)])
def test_sine_eigenvalues_every_mode(m, length):
    # The sine modes sin(j pi x / len), j = 1..m, are the eigenvectors of the
    # second-difference factor of A_h; every eigenvalue (not only j = 1) is pinned
    # against a dense symmetric eigensolver, and every mode against A_h itself.
    g = Grid((m,), (length,))
    A = laplacian(g).toarray()
    mu = sine_eigenvalues(m, g.h[0])
    assert np.allclose(np.sort(mu), np.linalg.eigvalsh(A), rtol=1e-11, atol=1e-9 * mu.max())
    x = g.coords(0)
    V = np.sin(np.pi * np.outer(x, np.arange(1, m + 1)) / length)
    assert np.max(np.abs(A @ V - V * mu[None, :])) <= 1e-10 * mu.max()


def test_sine_modes_of_the_box_laplacian():
    # Products of sine modes (x fastest) are eigenvectors of the 2D/3D A_h with the
    # sum of the axis eigenvalues, for low, high and mixed mode indices (the pairing
    # of mode index and eigenvalue index that the sampled-mode oracles rely on).
    rng = np.random.default_rng(7)
    for m in [(15, 9), (31, 20, 7), (63, 63)]:
        g = Grid(m)
        A = laplacian(g)
        mus = [sine_eigenvalues(mi, hi) for mi, hi in zip(g.m, g.h)]
        for _ in range(6):
            idx = [int(rng.integers(0, mi)) for mi in m]
            mode = np.ones(1)
            for a in range(g.dim):
                mode = np.kron(np.sin(np.pi * (idx[a] + 1) * g.coords(a)), mode)
            lam = sum(mus[a][idx[a]] for a in range(g.dim))
            assert np.max(np.abs(A @ mode - lam * mode)) <= 1e-10 * lam, (m, idx)


def test_refined_shifted_solve_is_exact_to_fp64():
    # Step 2 of the oracle's sweep against an independent extended-precision solution
    # in the sine basis (1D, m = 999: the shifted Laplacian's condition number is ~1e5).
    m, N = 999, 8
    g = Grid((m,))
    prob = Problem(laplacian(g), 2, 1.0, 0.5, N, 0.5, np.ones(m))
    rng = np.random.default_rng(3)
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    ld = np.longdouble
    pi = 4 * np.arctan(ld(1))
    j = np.arange(1, m + 1)
    S = np.sin(pi * (np.outer(j, j) % (2 * (m + 1))).astype(ld) / (m + 1))    # exact phase reduction
    mu = (4 * ld(m + 1) ** 2) * np.sin(pi * j.astype(ld) / (2 * (m + 1))) ** 2
    ta = ld(prob.tau) ** ld(prob.alpha)
    for p in (0, 1, N // 2):
        exact = (2 / ld(m + 1)) * (S @ ((S @ b.astype(np.clongdouble)) / (np.clongdouble(prob.d[p]) + ta * mu)))
        got = prob.shifted_solve(p, b)
        err = np.max(np.abs(got - exact.astype(np.complex128))) / np.max(np.abs(exact))
        assert err <= 1e-14, (p, err)


def test_eigenfunction_data_reduces_to_scalar_recurrence():
    # PIN-6: v = sin(pi x) sin(pi y) (x) ... and f = g(t) times the same mode give
    # U^n = y^n * mode with y^n the scalar scheme for mu = sum_i (4/h_i^2) sin^2(pi h_i/2).
    for m, k, alpha in [((9,), 3, 1.0), ((7, 5), 4, 1.0), ((5, 4, 3), 2, 0.6), ((6, 7), 5, 0.4)]:
        g = Grid(m)
        A = laplacian(g)
        mode = np.ones(1)
        for a in range(g.dim):
            mode = np.kron(np.sin(np.pi * g.coords(a)), mode)
        mu = sum(sine_eigenvalues(mi, hi)[0] for mi, hi in zip(g.m, g.h))
        N, T = 12, 0.7
        t = T * np.arange(N + 1) / N
        gt = np.cos(3 * t) + t ** 2
        # exact derivatives of g(t) = cos 3t + t^2 at 0: g' = 0, g'' = -9 + 2, g''' = 0, g'''' = 81
        fder, gd = None, None
        if k > 2:
            gd = [0.0, -7.0, 0.0, 81.0][:k - 2]
            fder = np.array(gd)[:, None] * mode[None, :]
        U = sequential(A, k, alpha, T, N, 2.0 * mode, np.outer(gt, mode), fder)
        y = sequential(np.array([[mu]]), k, alpha, T, N, np.array([2.0]), gt[:, None],
                       None if fder is None else np.array(gd)[:, None])
        assert np.max(np.abs(U - np.outer(y[:, 0], mode))) <= 1e-13 * np.max(np.abs(U))


CASES = [((15,), 16, 1.0, 1), ((15,), 16, 1.0, 2), ((15,), 16, 1.0, 3), ((15,), 16, 1.0, 4),
         ((15,), 16, 1.0, 5), ((15,), 16, 1.0, 6), ((15,), 16, 0.3, 2), ((15,), 16, 0.5, 3),
         ((15,), 16, 0.7, 6), ((7, 5), 16, 1.0, 4), ((7, 5), 16, 0.5, 1), ((3, 4, 5), 8, 1.0, 6),
         ((3, 4, 5), 8, 0.7, 2)]


@pytest.mark.parametrize("m,N,alpha,k", CASES)
def test_one_sweep_equals_dense_all_at_once_solve(m, N, alpha, k):
    # PIN-7: Algorithm 1/2 (O2, DFT diagonalization) == dense LU solve of P U = F (O3),
    # with F built from the kappa-circulant matrix itself, not from O2's sum.
    rng = np.random.default_rng(7)
    g = Grid(m)
    A = laplacian(g)
    M, T, kappa = g.M, 0.8, 0.05
    v = rng.standard_normal(M)
    f = rng.standard_normal((N + 1, M))
    fder = rng.standard_normal((k - 2, M)) if k > 2 else None
    Uprev = rng.standard_normal((N, M))
    tau = T / N
    B = kappa_circulant(k, alpha, N, kappa)
    L = lower_toeplitz(k, alpha, N)
    w = time_weights(k, alpha, N)
    s = np.cumsum(w)                       # s[n-1] = sum_{j<n} omega_j
    G = source_terms(A, k, alpha, T, N, v, f, fder) + tau ** (-alpha) * np.outer(s, v)
    F = G + tau ** (-alpha) * (np.kron(B - L, np.eye(M)) @ Uprev.reshape(-1)).reshape(N, M)
    ref = np.linalg.solve(all_at_once(A, k, alpha, T, N, kappa), F.reshape(-1)).reshape(N, M)
    prob = Problem(A, k, alpha, T, N, kappa, v, f, fder)
    for form in ("direct", "residual"):
        got, im = prob.sweep(Uprev, form)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref), form
        assert im <= 1e-12 * np.max(np.abs(ref))          # PIN-10 real-ness


@pytest.mark.parametrize("m,N,alpha,k", CASES[::3])
def test_sequential_is_the_fixed_point(m, N, alpha, k):
    # The time-stepping solution solves the lower block-triangular system (L (x) I)/tau^a + I (x) A
    # (the kappa-free part of the all-at-once matrix) with right-hand side G.
    rng = np.random.default_rng(11)
    g = Grid(m)
    A = laplacian(g).toarray()
    M, T = g.M, 0.8
    v = rng.standard_normal(M)
    f = rng.standard_normal((N + 1, M))
    fder = rng.standard_normal((k - 2, M)) if k > 2 else None
    tau = T / N
    s = np.cumsum(time_weights(k, alpha, N))
    G = source_terms(A, k, alpha, T, N, v, f, fder) + tau ** (-alpha) * np.outer(s, v)
    Tmat = tau ** (-alpha) * np.kron(lower_toeplitz(k, alpha, N), np.eye(M)) + np.kron(np.eye(N), A)
    ref = np.linalg.solve(Tmat, G.reshape(-1)).reshape(N, M)
    U = sequential(A, k, alpha, T, N, v, f, fder)
    assert np.linalg.norm(U - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("k,alpha,kappa", [(2, 1.0, 1e-3), (4, 1.0, 1e-5), (3, 0.5, 1e-4), (6, 1.0, 1e-2)])
def test_iteration_converges_to_sequential(k, alpha, kappa):
    # PIN-8: both forms reach the fixed point; the residual form to ~machine precision.
    w = wl.heat1d(m=31, N=32, k=k, kappa=kappa)
    g = Grid(w.m)
    A = laplacian(g)
    U = sequential(A, k, alpha, w.T, w.N, w.v, w.f, w.fder)
    prob = Problem(A, k, alpha, w.T, w.N, kappa, w.v, w.f, w.fder)
    Ur = iterate(prob, 6, init="v", form="residual")[-1]
    assert np.linalg.norm(Ur - U) <= 1e-12 * np.linalg.norm(U)
    Ud = iterate(prob, 6, init="v", form="direct")[-1]
    assert np.linalg.norm(Ud - U) <= 1e-9 * np.linalg.norm(U)


def test_roundoff_direct_vs_residual():
    # PIN-11 (trend): the direct form's floor grows as kappa shrinks (Sec. 2.2 roundoff
    # paragraph bounds it by C eps kappa^{-2} N^2); the residual form stays near eps.
    w = wl.heat1d(m=31, N=64, k=2)
    g = Grid(w.m)
    A = laplacian(g)
    U = sequential(A, 2, 1.0, w.T, w.N, w.v, w.f, w.fder)
    floors_d, floors_r = [], []
    for kappa in (1e-2, 1e-6):
        prob = Problem(A, 2, 1.0, w.T, w.N, kappa, w.v, w.f, w.fder)
        Ud = iterate(prob, 4, form="direct")[-1]
        Ur = iterate(prob, 4, form="residual")[-1]
        floors_d.append(np.linalg.norm(Ud - U) / np.linalg.norm(U))
        floors_r.append(np.linalg.norm(Ur - U) / np.linalg.norm(U))
    assert floors_d[1] > 10 * floors_d[0]
    assert max(floors_r) < 1e-13
    eps = np.finfo(float).eps
    assert floors_d[1] < 2.0 * eps * 64 ** 2 / 1e-6 ** 2      # within the paper's bound


def _thomas(a, b, c, r):
    """Unpivoted Thomas algorithm for a constant-coefficient tridiagonal system."""
    n = len(r)
    cp = np.zeros(n, dtype=complex)
    dp = np.zeros(n, dtype=complex)
    cp[0], dp[0] = c / b, r[0] / b
    for i in range(1, n):
        den = b - a * cp[i - 1]
        cp[i] = c / den
        dp[i] = (r[i] - a * dp[i - 1]) / den
    x = np.zeros(n, dtype=complex)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


@pytest.mark.parametrize("k,N,kappa,m", [(4, 512, 1e-5, 255), (6, 256, 1e-6, 127), (3, 1024, 1e-4, 511)])
def test_unpivoted_tridiagonal_is_stable_for_all_shifts(k, N, kappa, m):
    # PIN-12: for BDF >= 3 some shifts have Re d_p < 0, so the shifted systems are not
    # diagonally dominant.  Unpivoted elimination still matches pivoted LU on every shift.
    from oracle.sweep import eigenvalues
    alpha = 0.5 if k == 3 else 1.0
    d = eigenvalues(k, alpha, N, kappa)
    tau = 1.0 / N
    h = 1.0 / (m + 1)
    ta = tau ** alpha
    rng = np.random.default_rng(3)
    r = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    worst = 0.0
    for p in range(0, N // 2 + 1, max(1, N // 64)):
        for mux in (0.0, sine_eigenvalues(m, h)[-1]):      # y-systems after an x-DST
            b = d[p] + ta * (mux + 2.0 / h ** 2)
            a = -ta / h ** 2
            ab = np.zeros((3, m), dtype=complex)
            ab[0, 1:] = a
            ab[1, :] = b
            ab[2, :-1] = a
            ref = sla.solve_banded((1, 1), ab, r)
            got = _thomas(a, b, a, r)
            worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert worst < 1e-12


def test_sequential_exact_per_mode_on_long_lines():
    # O1 solves each step to FP64 rounding (long-double iterative refinement): on data
    # that are finite sine series, the trajectory equals the sum of the scalar schemes of
    # the modes (each sine is an eigenvector of A_h), here on the longest 1D line.  A plain
    # LU solve per step misses this by ~1e-11 at N = 2048.
    m, N, k = 2047, 512, 2
    w = wl.heat1d(seed=3, m=m, N=N, k=k, kappa=1e-3)
    g = Grid(w.m)
    U = sequential(laplacian(g), k, 1.0, w.T, N, w.v, w.f, w.fder)
    mu = sine_eigenvalues(m, g.h[0])
    idx = np.arange(1, m + 1)
    S = np.sin(np.pi * np.outer(idx, idx) / (m + 1))
    cv = S @ w.v * 2 / (m + 1)
    cf = (w.f @ S) * 2 / (m + 1)
    modes = np.nonzero(np.abs(cv) + np.abs(cf).max(axis=0) > 1e-12)[0]
    ref = np.zeros((N, m))
    for j in modes:
        y = sequential(mu[j], k, 1.0, w.T, N, np.array([cv[j]]), cf[:, j:j + 1])[:, 0]
        ref += np.outer(y, S[j])
    assert len(modes) == 8
    assert np.linalg.norm(U - ref) / np.linalg.norm(ref) <= 1e-12
    assert np.max(np.abs(U - ref)) <= 1e-12 * np.max(np.abs(ref))
