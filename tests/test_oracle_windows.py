"""Pins of the windowed oracle: one window is the sequential scheme itself, and
for BDF1 (no starting corrections, one-step history) restarting at a window's
end continues the global scheme exactly, so nwin windows of N steps equal one
solve of nwin N steps over the whole interval."""
import numpy as np

from oracle.grid import Grid, laplacian
from oracle.sequential import sequential
from oracle.windows import windowed_sequential
from paper_2007_13125_amd import workloads as wl


def test_one_window_is_the_sequential_scheme():
    w = wl.heat1d(seed=2, m=31, N=16, k=3)
    A = laplacian(Grid(w.m))
    ref = sequential(A, w.k, 1.0, w.T, w.N, w.v, w.f, w.fder)
    got = windowed_sequential(A, w.k, 1.0, w.T, w.N, 1, w.v, w.f, None if w.fder is None else w.fder[None])
    assert np.array_equal(got, ref)


def test_bdf1_windows_continue_the_global_scheme():
    nwin, N = 4, 8
    w = wl.heat1d(seed=3, m=31, N=nwin * N, k=1, T=2.0)
    A = laplacian(Grid(w.m))
    glob = sequential(A, 1, 1.0, w.T, nwin * N, w.v, w.f, None)
    win = windowed_sequential(A, 1, 1.0, w.T / nwin, N, nwin, w.v, w.f, None)
    assert np.max(np.abs(win - glob)) <= 1e-14 * np.max(np.abs(glob))


def test_bdf2_windows_restart_the_corrections():
    # with k >= 2 a restart is a different (still second-order) scheme: the windowed
    # trajectory departs from the global one after the first window only
    nwin, N = 3, 8
    w = wl.heat1d(seed=4, m=31, N=nwin * N, k=2, T=1.5)
    A = laplacian(Grid(w.m))
    glob = sequential(A, 2, 1.0, w.T, nwin * N, w.v, w.f, None)
    win = windowed_sequential(A, 2, 1.0, w.T / nwin, N, nwin, w.v, w.f, None)
    assert np.array_equal(win[:N], glob[:N])
    assert np.max(np.abs(win[N:] - glob[N:])) > 1e-8
