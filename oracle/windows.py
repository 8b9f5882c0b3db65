"""Windowed time stepping (oracle; test infrastructure).

The remark that closes Sec. 4's Example 4 proposes time windows: a number of
steps is computed (in parallel) in the current window, and the computation is
restarted for the next window sequentially.  The result of a windowed solve
is therefore the corrected scheme restarted at every window: window w solves
the N-step scheme on its own interval of length T with initial value the last
level of window w-1 (v for the first) and the Table 1 corrections built from f
and its derivatives at the window's start.  This module computes that with
the sequential oracle (O1), window after window.
"""
import numpy as np

from .sequential import sequential


def windowed_sequential(A, k, alpha, T, N, nwin, v, f=None, fder=None):
    """U^1..U^{nwin N} as [nwin N, M].  f: [nwin N + 1, M] or None; fder:
    [nwin, k-2, M] (derivatives at each window's start) or None."""
    M = A.shape[0]
    out = np.zeros((nwin * N, M))
    vw = np.asarray(v, dtype=np.float64)
    for w in range(nwin):
        fw = None if f is None else f[w * N:w * N + N + 1]
        dw = None if (fder is None or k <= 2) else fder[w]
        Uw = sequential(A, k, alpha, T, N, vw, fw, dw)
        out[w * N:(w + 1) * N] = Uw
        vw = Uw[-1]
    return out
