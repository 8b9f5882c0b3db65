"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
binding and the CPU oracle on the same seeded workload."""
import numpy as np

from oracle.fem import FemProblem, fem_sequential
from oracle.grid import Grid, laplacian
from oracle.sequential import sequential
from oracle.sweep import Problem, iterate


def space_of(w):
    return getattr(w, "space", "fd")


def to_dev(a):
    import torch
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_solve(w, precision="fp64", form="residual", init="v", tol=None, max_sweeps=40, norm="inf", variants=None):
    import torch

    from paper_2007_13125_amd.binding import Plan
    print(f"[gpu] solve {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha} kappa={w.kappa} "
          f"{precision}/{form}/{init}/{space_of(w)} variants={variants}", flush=True)
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=tol or w.tol, max_sweeps=max_sweeps,
                precision=precision, form=form, init=init, norm=norm, space=space_of(w))
    if variants is not None:
        plan.set_variants(variants)
    U, info = plan.solve(to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    torch.cuda.synchronize()
    out = U.cpu().numpy()
    plan.close()
    return out, info


def gpu_iterates(w, sweeps, precision="fp64", form="residual", init="v"):
    """U_0 .. U_sweeps from the GPU, one pint_sweeps call per sweep."""
    import torch

    from paper_2007_13125_amd.binding import Plan
    print(f"[gpu] iterates {w.name} m={w.m} N={w.N} k={w.k} alpha={w.alpha} {precision}/{form}/{space_of(w)}",
          flush=True)
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, precision=precision, form=form, init=init,
                space=space_of(w))
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
    N = N or w.N
    T = T or w.T
    f = None if w.f is None else w.f[:N + 1]
    if space_of(w) == "fem":
        return fem_sequential(w.m[0], w.k, w.alpha, T, N, w.v, f, w.fder)
    A = laplacian(Grid(w.m))
    return sequential(A, w.k, w.alpha, T, N, w.v, f, w.fder)


def oracle_iterates(w, sweeps, form="residual", init="v"):
    if space_of(w) == "fem":
        prob = FemProblem(w.m[0], w.k, w.alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    else:
        prob = Problem(laplacian(Grid(w.m)), w.k, w.alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    return iterate(prob, sweeps, init=init, form=form)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """Element-wise check beside rel_l2: the largest entry error relative to the
    largest reference entry (an error confined to a few entries is not diluted
    by the size of the array)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def errors(a, b):
    return rel_l2(a, b), max_rel(a, b)


def oracle_modal(w, dofs):
    """Sequential oracle in sine-mode space for data that is a finite sine series.

    The sampled sines are exact eigenvectors of A_h (pinned by the eigenfunction
    test of the oracle), so each mode evolves by the scalar scheme with
    mu = sum_a (4/h_a^2) sin^2((i_a+1) pi h_a/2); the trajectory is assembled at
    the requested dofs only.  Returns [N, len(dofs)]."""
    import scipy.sparse as sp

    from oracle.grid import sine_eigenvalues
    from paper_2007_13125_amd.workloads import _cos_profile_derivs

    g = Grid(w.m)
    cv, cf = w.modes["v"], w.modes["f"]
    shape = cv.shape
    mus = [sine_eigenvalues(g.m[a], g.h[a])[:shape[a]] for a in range(g.dim)]
    grids = np.meshgrid(*mus, indexing="ij")
    mu = sum(grids).reshape(-1)
    f, fder = _cos_profile_derivs(w.N, w.T, w.k, cf.reshape(-1))
    C = sequential(sp.diags(mu), w.k, w.alpha, w.T, w.N, cv.reshape(-1), f, fder)
    # basis values at the sampled dofs (x fastest ordering)
    dofs = np.asarray(dofs)
    coords = []
    rem = dofs.copy()
    for a in range(g.dim):
        coords.append(rem % g.m[a])
        rem = rem // g.m[a]
    phi = np.ones((C.shape[1], len(dofs)))
    idx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    for a in range(g.dim):
        ia = idx[a].reshape(-1)
        phi *= np.sin(np.pi * np.outer(ia + 1, coords[a] + 1) / (g.m[a] + 1))
    return C @ phi
