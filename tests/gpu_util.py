"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
binding and the CPU oracle on the same seeded workload."""
import numpy as np

from oracle.grid import Grid, laplacian
from oracle.sequential import sequential
from oracle.sweep import Problem, iterate


def to_dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_solve(w, precision="fp64", form="residual", init="v", tol=None, max_sweeps=40, norm="inf"):
    import torch

    from paper_2007_13125_amd.binding import Plan
    print(f"[gpu] solve {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha} kappa={w.kappa} "
          f"{precision}/{form}/{init}", flush=True)
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=tol or w.tol, max_sweeps=max_sweeps,
                precision=precision, form=form, init=init, norm=norm)
    U, info = plan.solve(to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    plan.close()
    return out, info


def gpu_iterates(w, sweeps, precision="fp64", form="residual", init="v"):
    """U_0 .. U_sweeps from the GPU, one pint_sweeps call per sweep."""
    import torch

    from paper_2007_13125_amd.binding import Plan
    print(f"[gpu] iterates {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha} {precision}/{form}", flush=True)
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, precision=precision, form=form, init=init)
    U = torch.empty((w.N, int(np.prod(w.m))), dtype=torch.float64, device="cuda")
    v, f, fd = to_dev(w.v), to_dev(w.f), to_dev(w.fder)
    plan.bind(v, f, fd)
    plan.init_iterate(U)
    out = [U.cpu().numpy()]
    norms = torch.zeros((sweeps, 2), dtype=torch.float64, device="cuda")
    for s in range(sweeps):
        plan.sweeps(U, 1, norms[s])
        out.append(U.cpu().numpy())
    torch.cuda.synchronize()
    nrm = norms.cpu().numpy()
    plan.close()
    return out, nrm


def oracle_solution(w, N=None, T=None):
    A = laplacian(Grid(w.m))
    N = N or w.N
    T = T or w.T
    f = None if w.f is None else w.f[:N + 1]
    return sequential(A, w.k, w.alpha, T, N, w.v, f, w.fder)


def oracle_iterates(w, sweeps, form="residual", init="v"):
    A = laplacian(Grid(w.m))
    prob = Problem(A, w.k, w.alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    return iterate(prob, sweeps, init=init, form=form)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
