"""CPU model of the index scheme of the sine passes with the odd extension
folded into the first and last FFT stages (k_dst_colsf for y/z columns,
k_dst_rowsf for x rows; they differ only in the LDS layout of a line): the same
butterfly, partner and position formulas, applied with plain numpy DFTs, must
give the raw sine transform -2i S x (S_kt = sin(pi k t/(m+1))) and, for the
solve pass, the raw transform of the divided transform.  This pins the folding
arithmetic (which half of which butterfly feeds which stage) independently of
the GPU."""
import numpy as np
import pytest


def _radix0(logl):
    return {8: 16, 9: 8, 10: 16, 11: 16}[logl]


def _dft(v):
    n = np.arange(len(v))
    return np.exp(-2j * np.pi * np.outer(n, n) / len(v)) @ v


def _stockham_stage(buf, L, rad, W, ns):
    """Generic Stockham stage (span ns): butterfly j reads x[j + r L/rad], twiddles
    w^{r k L/(rad ns)} (k = j mod ns), and writes (j - k) rad + k + r ns."""
    q = L // rad
    out = np.empty_like(buf)
    for j in range(q):
        k = j % ns
        tw = np.exp(-2j * np.pi * np.arange(rad) * k * (q // ns) / L)
        for b in range(W):
            v = _dft(buf[[(j + r * q) * W + b for r in range(rad)]] * tw)
            for r in range(rad):
                out[((j - k) * rad + k + r * ns) * W + b] = v[r]
    return out


def _folded_transform(nat, L, W):
    """One raw transform of odd columns given in natural layout nat[k W + b],
    k = 0..L/2 (k = 0 and L/2 zero); returns the lower halves Y[(j, b)] =
    (Y_{j + Q r}, r < R0/2) of the last stage's butterflies."""
    logl = L.bit_length() - 1
    R0 = _radix0(logl)
    Q, H = L // R0, R0 // 2
    lmid = logl - 2 * (R0.bit_length() - 1)
    buf = np.zeros(L * W, complex)
    for j in range(Q):                       # first stage (span 1)
        for b in range(W):
            v = np.zeros(R0, complex)
            for s in range(H):
                v[s] = nat[(j + Q * s) * W + b]
                v[R0 - 1 - s] = -nat[((Q - j) + Q * s) * W + b]
            v = _dft(v)
            for r in range(R0):
                buf[(j * R0 + r) * W + b] = v[r]
    if lmid:
        buf = _stockham_stage(buf, L, 1 << lmid, W, R0)
    Y = {}
    for j in range(Q):                       # last stage (span Q), lower half kept
        tw = np.exp(-2j * np.pi * np.arange(R0) * j / L)
        for b in range(W):
            Y[(j, b)] = _dft(buf[[(j + Q * r) * W + b for r in range(R0)]] * tw)[:H]
    return Y, Q, H


def _fold_pass(x, c=None):
    m, W = x.shape
    L = 2 * (m + 1)
    nat = np.zeros((L // 2 + 1) * W, complex)
    nat[W:(m + 1) * W] = x.reshape(-1)       # x_t at position t = 1..m
    Y, Q, H = _folded_transform(nat, L, W)
    if c is not None:                        # divide, then the same transform again
        nat = np.zeros((L // 2 + 1) * W, complex)
        for (j, b), v in Y.items():
            for r in range(H):
                k = j + Q * r
                if 1 <= k <= m:
                    nat[k * W + b] = v[r] * c[k - 1, b]
        Y, Q, H = _folded_transform(nat, L, W)
    out = np.zeros((m, W), complex)
    for (j, b), v in Y.items():
        for r in range(H):
            k = j + Q * r
            if 1 <= k <= m:
                out[k - 1, b] = v[r]
    return out


@pytest.mark.parametrize("logl", [8, 9, 10, 11])
def test_folded_schedule_gives_the_sine_transform(logl):
    rng = np.random.default_rng(logl)
    m, W = (1 << logl) // 2 - 1, 3
    x = rng.standard_normal((m, W)) + 1j * rng.standard_normal((m, W))
    S = np.sin(np.pi * np.outer(np.arange(1, m + 1), np.arange(1, m + 1)) / (m + 1))
    ref = -2j * (S @ x)
    got = _fold_pass(x)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    c = rng.standard_normal((m, W)) + 1j * rng.standard_normal((m, W))
    ref2 = -2j * (S @ (c * ref))
    got2 = _fold_pass(x, c)
    assert np.abs(got2 - ref2).max() <= 1e-12 * np.abs(ref2).max()
