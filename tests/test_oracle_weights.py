"""Pins of the oracle's time weights and eigenvalues against facts fixed
outside the oracle: textbook BDF coefficients, order conditions, the k = 1
binomial closed form of the CQ weights, an independent Cauchy-integral
evaluation of the power series, and the closed-form eigenvalues
delta_k(kappa^{1/N} e^{-2 pi i p/N}) used in Sec. 2.2's roundoff analysis."""
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import binom

from oracle.bdf import bdf_weights, table1_a, table1_b
from oracle.bruteforce import kappa_circulant
from oracle.cq import cq_weights, time_weights
from oracle.sweep import eigenvalues

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _textbook():
    rows = {}
    with open(os.path.join(GOLDEN, "bdf_textbook.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, vals = line.split(":")
            rows[int(k)] = [Fraction(x) for x in vals.split()]
    return rows


@pytest.mark.parametrize("k", range(1, 7))
def test_bdf_weights_match_textbook(k):
    # PIN-1: Sec. 2.1 eq. bdf-gen gives the classical BDF coefficients.
    assert bdf_weights(k) == _textbook()[k]


@pytest.mark.parametrize("k", range(1, 7))
def test_bdf_order_conditions(k):
    # delta_k(e^{-z}) = z + O(z^{k+1}): sum_j omega_j (-j)^p / p! = [p == 1], p = 0..k.
    w = bdf_weights(k)
    for p in range(0, k + 1):
        s = sum(wj * Fraction(-j) ** p for j, wj in enumerate(w))
        assert s == (1 if p == 1 else 0), (k, p)
    # omega_0 is the harmonic number H_k.
    assert w[0] == sum(Fraction(1, l) for l in range(1, k + 1))


def test_table1_structure():
    # Table 1 holds k-1 values a_n and a (k-2) x (k-1) block b_{l,n}; all vanish for n >= k.
    for k in range(1, 7):
        for n in range(k, k + 3):
            assert table1_a(k, n) == 0
            for l in range(1, 5):
                assert table1_b(k, l, n) == 0
    assert table1_a(2, 1) == Fraction(1, 2)
    assert table1_b(6, 3, 1) == Fraction(-1, 360)


@pytest.mark.parametrize("alpha", [0.1, 0.3, 0.5, 0.7, 0.9])
def test_cq_weights_k1_binomial(alpha):
    # PIN-2: for BDF1, delta_1(xi)^alpha = (1 - xi)^alpha, omega_n = (-1)^n binom(alpha, n)
    # (Lemma 3.1's closed form, with the sign read as + prod (1 - (1+alpha)/j)).
    n = np.arange(400)
    ref = (-1.0) ** n * binom(alpha, n)
    got = cq_weights(1, alpha, 400)
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
    prod = np.cumprod(np.concatenate([[1.0], 1.0 - (1.0 + alpha) / np.arange(1, 400)]))
    assert np.allclose(got, prod, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("k", range(1, 7))
def test_cq_weights_alpha_one_are_bdf(k):
    w = cq_weights(k, 1.0, 40)
    ref = np.zeros(40)
    ref[:k + 1] = [float(x) for x in bdf_weights(k)]
    assert np.max(np.abs(w - ref)) <= 1e-13
    assert np.array_equal(time_weights(k, 1.0, 40), ref)


@pytest.mark.parametrize("k", range(1, 7))
@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_cq_weights_cauchy_integral(k, alpha):
    # Independent route ("by FFT", Sec. 3.1): sample delta_k(xi)^alpha on |xi| = r with the
    # principal branch (delta_k maps the disc into a sector avoiding the negative axis for
    # k <= 6, Lemma 2.1) and read off the Taylor coefficients with an FFT.
    K, r, n = 8192, 0.97, 64
    xi = r * np.exp(2j * np.pi * np.arange(K) / K)
    delta = sum((1.0 - xi) ** l / l for l in range(1, k + 1))
    c = np.fft.fft(delta ** alpha) / K
    ref = (c[:n] / r ** np.arange(n)).real
    got = cq_weights(k, alpha, n)
    assert np.max(np.abs(got - ref)) <= 1e-12


@pytest.mark.parametrize("k", [1, 3, 6])
@pytest.mark.parametrize("alpha", [0.3, 0.7])
def test_cq_weights_decay(k, alpha):
    # Lemma 3.1: |omega_n| <= c (n+1)^{-alpha-1}; the scaled weights stay bounded and,
    # for large n, approach a constant (the decay exponent is exactly -1-alpha).
    w = cq_weights(k, alpha, 4001)
    n = np.arange(4001)
    scaled = np.abs(w) * (n + 1.0) ** (1.0 + alpha)
    tail = scaled[1000:]
    assert tail.max() / tail.min() < 1.05
    assert np.all(scaled[1:] < 25.0)
    # the weights sum to delta_k(1)^alpha = 0: partial sums decay like n^{-alpha}
    s = np.cumsum(w)
    r = (s[3999] * 4000.0 ** alpha) / (s[999] * 1000.0 ** alpha)
    assert abs(r - 1.0) < 0.05


@pytest.mark.parametrize("k", [2, 4, 6])
@pytest.mark.parametrize("N", [16, 100])
def test_diagonalization_identity(k, N):
    # PIN-3: B_k(kappa) = Lambda V diag(d) V^{-1} Lambda^{-1} (Lemma diag-heat), and for
    # BDF-k the eigenvalues are delta_k(kappa^{1/N} e^{-2 pi i p/N}) (Sec. 2.2, roundoff).
    kappa = 0.1
    B = kappa_circulant(k, 1.0, N, kappa)
    d = eigenvalues(k, 1.0, N, kappa)
    q = np.arange(N)
    Lam = np.diag(kappa ** (-q / N))
    V = np.exp(2j * np.pi * np.outer(q, q) / N)
    rebuilt = Lam @ V @ np.diag(d) @ np.linalg.inv(V) @ np.linalg.inv(Lam)
    assert np.max(np.abs(rebuilt - B)) <= 1e-12 * np.max(np.abs(B))
    zeta = kappa ** (1.0 / N) * np.exp(-2j * np.pi * q / N)
    closed = sum((1.0 - zeta) ** l / l for l in range(1, k + 1))
    assert np.max(np.abs(d - closed)) <= 1e-12 * np.max(np.abs(closed))


@pytest.mark.parametrize("alpha", [0.3, 0.5])
def test_cq_eigenvalues_match_dense_eigensolver(alpha):
    N, k, kappa = 24, 3, 0.05
    B = kappa_circulant(k, alpha, N, kappa)
    ev = np.linalg.eigvals(B)
    d = eigenvalues(k, alpha, N, kappa)
    # match as multisets
    for lam in d:
        assert np.min(np.abs(ev - lam)) <= 1e-10 * np.max(np.abs(d))


@pytest.mark.parametrize("k,alpha", [(2, 1.0), (5, 1.0), (3, 0.5)])
def test_eigenvalues_hermitian_pairs(k, alpha):
    # PIN-10 (part): real weights give d_{N-p} = conj(d_p), so half the spectrum suffices.
    N = 64
    d = eigenvalues(k, alpha, N, 1e-3)
    assert np.max(np.abs(d[1:][::-1] - np.conj(d[1:]))) <= 1e-13 * np.max(np.abs(d))
    assert abs(d[0].imag) < 1e-13 and abs(d[N // 2].imag) < 1e-13
