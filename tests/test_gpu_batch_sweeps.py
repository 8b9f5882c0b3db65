"""Batched sweeps of 1D problems (every pass of a sweep one launch over all
active problems of a class, a host stop test per problem after each sweep): a
batch of problems with different m, N (powers of two and others), k, alpha,
kappa and precision, each against the sequential oracle, through
pint_batch_plan_create / pint_batch_solve; and a batch that mixes 1D, 2D and
3D problems (the 2D and 3D ones take the single-plan path and must equal their
own single-plan solves bit for bit)."""
import numpy as np
import pytest

from paper_2007_13125_amd import binding as B
from paper_2007_13125_amd import workloads as wl
from tests.gpu_util import errors, gpu_solve, oracle_solution, to_dev

pytestmark = pytest.mark.gpu


def _batch(ws, precs, tol=1e-13, max_sweeps=40):
    import torch
    grids = [B.make_grid(w.m) for w in ws]
    params = [B.make_params(w.k, w.alpha, w.T, w.N, w.kappa, tol=tol, max_sweeps=max_sweeps, precision=p)
              for w, p in zip(ws, precs)]
    print("[gpu] batch:", [(w.m, w.N, w.k, w.alpha, p) for w, p in zip(ws, precs)], flush=True)
    h = B.pint_batch_plan_create(grids, params)
    data = [(to_dev(w.v), to_dev(w.f), to_dev(w.fder)) for w in ws]
    Us = [torch.empty((w.N, w.M), dtype=torch.float64, device="cuda") for w in ws]
    st, upd, sw = B.pint_batch_solve(h, [d[0] for d in data], [d[1] for d in data], [d[2] for d in data], Us,
                                     max_sweeps)
    torch.cuda.synchronize()
    B.pint_plan_destroy(h)
    return st, [U.cpu().numpy() for U in Us], upd, sw


def test_1d_batch_matches_oracle():
    ws = [wl.heat1d(seed=41, m=63, N=64, k=2, kappa=1e-3), wl.heat1d(seed=42, m=100, N=32, k=5, kappa=1e-2),
          wl.heat1d(seed=43, m=255, N=128, k=3, kappa=1e-3), wl.heat1d(seed=44, m=31, N=100, k=4, kappa=1e-2),
          wl.heat1d(seed=45, m=500, N=16, k=6, kappa=1e-4), wl.heat1d(seed=46, m=7, N=6, k=1, kappa=0.1)]
    ws[2].alpha = 0.5
    ws[3].alpha = 0.7
    precs = ["fp64", "mixed", "fp64", "fp64", "mixed", "fp64"]
    st, got, upd, sw = _batch(ws, precs)
    assert st == B.PINT_OK, (st, sw)
    for i, (w, p) in enumerate(zip(ws, precs)):
        err = errors(got[i], oracle_solution(w))
        print(f"instance {i}: m={w.m} N={w.N} k={w.k} alpha={w.alpha} {p}: sweeps={sw[i]} upd={upd[i][-2:]} "
              f"(rel_l2, max_rel)={err}", flush=True)
        assert max(err) <= (1e-11 if p == "fp64" else 1e-10), (i, err)
        assert upd[i][-1] <= 1e-13 and 1 <= sw[i] < 40


def test_batch_of_recipe_1d_instances():
    # 1D instances of the many-instance recipe (m 63..1023, N 32..1024, k 1..6,
    # alpha in {1, 0.3, 0.7}, kappa 1e-6..1e-2), mixed precision, stop test 1e-10
    ws, i = [], 0
    while len(ws) < 8:
        w = wl.batch_instance(i)
        if len(w.m) == 1 and w.N * w.M <= 2 ** 18:
            ws.append(w)
        i += 1
    st, got, upd, sw = _batch(ws, ["mixed"] * len(ws), tol=1e-10)
    assert st == B.PINT_OK, (st, sw)
    for i, w in enumerate(ws):
        err = errors(got[i], oracle_solution(w))
        print(f"recipe 1D {i}: m={w.m} N={w.N} k={w.k} alpha={w.alpha} kappa={w.kappa:.2g}: sweeps={sw[i]} "
              f"(rel_l2, max_rel)={err}", flush=True)
        assert max(err) <= 1e-10, (i, err)


def test_batch_of_mixed_dimensions():
    ws = [wl.heat1d(seed=51, m=63, N=64, k=2, kappa=1e-3), wl.heat2d(seed=52, m=(31, 15), N=128, k=4, kappa=1e-4),
          wl.heat1d(seed=53, m=127, N=48, k=3, kappa=1e-3), wl.heat3d(seed=54, m=(7, 15, 7), N=32, k=6, kappa=1e-4),
          wl.heat2d(seed=55, m=(20, 33), N=30, k=3, kappa=1e-3), wl.heat1d(seed=56, m=40, N=256, k=4, kappa=1e-4),
          wl.heat1d(seed=57, m=50, N=2048, k=2, kappa=1e-3), wl.heat1d(seed=58, m=33, N=1500, k=3, kappa=1e-3)]
    ws[2].alpha = 0.6
    ws[4].alpha = 0.5
    ws[6].alpha = 0.5   # the 4096-point history convolution, power-of-two time DFTs
    ws[7].alpha = 0.4   # the same convolution, Bluestein time DFTs
    precs = ["fp64", "fp64", "mixed", "mixed", "fp64", "fp64", "fp64", "mixed"]
    st, got, upd, sw = _batch(ws, precs)
    assert st == B.PINT_OK, (st, sw)
    for i, (w, p) in enumerate(zip(ws, precs)):
        err = errors(got[i], oracle_solution(w))
        print(f"mixed-dim {i}: m={w.m} N={w.N} k={w.k} alpha={w.alpha} {p}: sweeps={sw[i]} (rel_l2, max_rel)={err}",
              flush=True)
        assert max(err) <= (1e-11 if p == "fp64" else 1e-10), (i, err)
        if len(w.m) > 1:
            single, info = gpu_solve(w, precision=p, tol=1e-13, max_sweeps=40)
            assert info["sweeps"] == sw[i] and np.array_equal(got[i], single), i
            assert upd[i] == list(info["upd"][:sw[i]]), i
