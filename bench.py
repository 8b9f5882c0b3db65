"""Benchmark of the diagonalized waveform-relaxation sweep on one MI355X.

One step = one whole WR sweep (residual + kappa scaling + forward time FFT,
spatial shifted solves, inverse time FFT + unscale + update + norms).  The
headline workload is the largest one that fits one GPU: 3D heat, 7-point FD
Dirichlet Laplacian on 127^3 interior nodes, BDF6, T = 1, N = 256,
kappa = 1e-6, seeded smooth sine-series data (5.2e8 space-time unknowns).
Inputs are resident in HBM before the timed region.

Prints ONE JSON line: the FP64 sweep throughput (space-time unknown-updates
per second) as `value`; the mixed FP32/FP64 and FP64 direct-form sweeps
alongside; per-launch device times from HIP events recorded on the plan's
stream inside the timed region (repeated passes listed in launch order and
summed per pass name); the HBM roofline of the dominant kernel; time-to-1e-10
against the FP64 CPU oracle for FP64 residual, FP64 direct and mixed; the
sequential-in-time GPU solver's time to the same trajectory; the same figures
for the 2D heat (255^2 x 512, BDF4) and 2D subdiffusion (511^2 x 1024, CQ-BDF3)
workloads; sweeps/s and time-to-1e-12 of the 1D heat workload (63 x 64, BDF2);
the many-instance batch; wall-clock times of Algorithm 3, P1 elements and
windowed solves (`next_rows`); and the CPU oracle timed on a bounded sample.
"""
import argparse
import glob
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "space-time unknown-updates/s per WR sweep + time-to-1e-10, FP64 vs mixed; %HBM"
HBM_PEAK_GBS = 8000.0
HEADLINE = "heat3d"
SWEEP_WORKLOADS = ("heat3d", "heat2d", "subdiff2d")
KERNEL_SOURCES = ["paper_2007_13125_amd/csrc/pint_device.h", "paper_2007_13125_amd/csrc/pint_forward.hip",
                  "paper_2007_13125_amd/csrc/pint_space.hip", "paper_2007_13125_amd/csrc/pint_time.hip"]
COPY_BYTES = 256 << 20
DESCR = {
    "heat3d": "3D heat, 7-point FD Dirichlet Laplacian 127^3, BDF6 (Table 1 corrections), T=1, N=256, kappa=1e-6",
    "heat2d": "2D heat, 5-point FD Dirichlet Laplacian 255^2, BDF4 (Table 1 corrections), T=1, N=512, kappa=1e-5",
    "subdiff2d": "2D subdiffusion, Caputo alpha=1/2, CQ-BDF3, 5-point FD 511^2, T=1, N=1024, kappa=1e-4, f=0, "
                 "indicator + noise initial value",
    "heat1d": "1D heat, 3-point FD m=63, BDF2, T=1, N=64, kappa=1e-3",
}


def profile_stem(w):
    dims = "x".join(str(m) for m in w.m)
    tag = f"bdf{w.k}" if w.alpha == 1.0 else f"cqbdf{w.k}"
    return os.path.join(ROOT, "profiles", f"{w.name}_{dims}_N{w.N}_{tag}")


def sources_sha():
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()


# ---------------------------------------------------------------------------------------
# algorithmic bytes

def spectrum_bytes(N, M, mixed):
    return (N // 2 + 1) * M * (8 if mixed else 16)


def slot_bytes(name, w, mixed):
    """Algorithmic HBM bytes of one launch of a pass (each array read or written once)."""
    N, M = w.N, w.M
    S = spectrum_bytes(N, M, mixed)
    if name.startswith("forward"):
        return 8 * N * M + (8 * N * M if w.f is not None else 0) + 8 * M + S   # U, f, v in; spectrum out
    if name == "direct_rhs_spectrum":
        return 2 * S + 8 * w.k * M                                            # source spectrum, k rows of U
    if name.startswith("inverse"):
        return S + 16 * N * M                                                 # spectrum in; U in and out
    if name == "norm_reduce":
        return 0
    return 2 * S                                                              # spatial pass: in place


def three_stage_bytes(w, mixed):
    """The method's floor with its two time <-> space transposes: U, f in, U out, and
    the half spectrum written and read twice (24 + 4c bytes per unknown, c = bytes per
    half-spectrum value per unknown; 16 + 4c when f = 0)."""
    N, M = w.N, w.M
    return 8 * N * M * (3 if w.f is not None else 2) + 2 * spectrum_bytes(N, M, mixed)


def measured_traffic(w, precision, slot, variants):
    """HBM bytes per launch of a pass from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record of this workload, or None when that record is missing, was
    taken with other kernel variants, or the kernel sources changed since."""
    try:
        rec = json.load(open(profile_stem(w) + "_traffic.json"))
        if rec["sources_sha256"] != sources_sha() or list(rec.get("variants", [])) != list(variants):
            return None
        k = rec["kernels"][precision][slot]
        return k["read"] + k["write"]
    except (OSError, KeyError, ValueError):
        return None


def profiled_kernels(w, precision, slot):
    """The kernel(s) that make up a pass in the committed profile record, or None."""
    try:
        return json.load(open(profile_stem(w) + "_traffic.json"))["kernels"][precision][slot]["kernel"]
    except (OSError, KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------------------
# GPU runs

def to_dev(a):
    import torch
    return None if a is None else torch.from_numpy(a).to("cuda")


def run_variant(w, precision, form, steps, warmup, tune):
    """Plan + bound data + a U; the timed region is `steps` sweeps with a HIP event
    pair around every launch on the plan's stream.  Returns (plan, U, ms_per_step,
    slots [(pass, ms per launch)] in launch order, variants)."""
    import torch

    from paper_2007_13125_amd.binding import Plan
    data = (to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-14, max_sweeps=30, precision=precision, form=form)
    plan.bind(*data)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    plan.init_iterate(U)
    # kernel variants chosen by the library's autotuner (plan setup, outside the timed region)
    variants = plan.tune(U, 3) if tune else plan.variants()
    plan.init_iterate(U)
    if warmup:
        plan.sweeps(U, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slots = plan.profile(U, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return plan, U, (t1 - t0) / steps * 1e3, slots, variants


def slot_summary(slots):
    by = {}
    for n, t in slots:
        by[n] = by.get(n, 0.0) + t
    return {"launches": [[n, t] for n, t in slots], "per_pass": by}


def roofline_of(w, precision, slots, variants):
    mixed = precision == "mixed"
    dom = max(slots, key=lambda s: s[1])
    b = slot_bytes(dom[0], w, mixed)
    gbs = b / (dom[1] * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom[0], "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(w, precision, dom[0], variants), "alg_bytes": b,
            "ms": dom[1], "launches": profiled_kernels(w, precision, dom[0])}


def sampler(w):
    """GPU-side sample of a trajectory that the oracle evaluates one by one: the
    values at 4096 seeded dofs (heat: the data are finite sine series), or the
    coefficients of 16 x 16 sine modes of every level (subdiffusion), or the whole
    trajectory (1D heat)."""
    import numpy as np
    import torch
    if w.name == "heat1d":
        return None, (lambda U: U.cpu().numpy())
    if w.name == "subdiff2d":
        mx, my = w.m
        sx = np.sin(np.pi * np.outer(np.arange(1, mx + 1), MODE_IDX + 1) / (mx + 1))
        sy = np.sin(np.pi * np.outer(np.arange(1, my + 1), MODE_IDX + 1) / (my + 1))
        tx, ty = to_dev(sx), to_dev(sy)
        c = 4.0 / ((mx + 1) * (my + 1))

        def proj(U):
            a = U.view(w.N, my, mx) @ tx                            # [N, y, i]
            return (c * (a.transpose(1, 2) @ ty)).reshape(w.N, -1).cpu().numpy()
        return None, proj
    dofs = np.random.default_rng(0).choice(w.M, 4096, replace=False)
    di = torch.from_numpy(dofs).to("cuda")
    return dofs, (lambda U: U.index_select(1, di).cpu().numpy())


MODE_IDX = None  # set in main (numpy array of sampled sine-mode indices, 0-based)


def time_to_tol(plan, U, sample, ref, tol, max_sweeps=12):
    """Sweeps m* until the sampled trajectory is within tol (relative L2) of the
    oracle, found in an untimed validation run with a snapshot after every sweep;
    then the wall time of exactly m* sweeps from U_0 (best of three)."""
    import numpy as np
    import torch
    plan.init_iterate(U)
    nref = np.linalg.norm(ref)
    mstar, errs = None, []
    for s in range(1, max_sweeps + 1):
        plan.sweeps(U, 1)
        e = float(np.linalg.norm(sample(U) - ref) / nref)
        errs.append(e)
        if e <= tol:
            mstar = s
            break
    out = {"sweeps": mstar, "ms": None, "rel_l2_per_sweep": [float("%.3g" % e) for e in errs]}
    if mstar is not None:
        best = float("inf")
        for _ in range(3):
            plan.init_iterate(U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.sweeps(U, mstar)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        out["ms"] = best * 1e3
    return out


def bench_workload(w, args, refs):
    import torch
    entry = {"workload": DESCR[w.name], "grid": list(w.m), "N": w.N, "k": w.k, "alpha": w.alpha,
             "kappa": w.kappa, "unknowns": w.N * w.M}
    dofs, sample = sampler(w)
    for precision, form in (("fp64", "residual"), ("mixed", "residual"), ("fp64", "direct")):
        key = precision if form == "residual" else "fp64_direct"
        print(f"[bench] {w.name} {key}", file=sys.stderr, flush=True)
        plan, U, ms, slots, var = run_variant(w, precision, form, args.steps, args.warmup, not args.no_tune)
        mixed = precision == "mixed"
        asb = sum(slot_bytes(n, w, mixed) for n, _ in slots)
        e = {"ms_per_step": ms, "value": w.N * w.M / (ms * 1e-3), "kernels_ms": slot_summary(slots),
             "hbm_frac_as_built": asb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "hbm_frac_3stage": three_stage_bytes(w, mixed) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
             "roofline": roofline_of(w, precision, slots, var), "variants": var}
        if refs is not None and w.name in refs:
            e["time_to_1e-10"] = time_to_tol(plan, U, sample, refs[w.name], 1e-10)
        entry[key] = e
        plan.close()
        del U
        torch.cuda.empty_cache()
    if not args.only:
        entry["sequential"] = sequential_time(w)
    return entry


def sequential_time(w, reps=2):
    """Wall time of the sequential-in-time GPU solver (the scheme stepped level by
    level, one shifted spatial solve per step), FP64: the in-GPU baseline the
    parallel-in-time sweeps are compared with (time to the same trajectory)."""
    import torch

    from paper_2007_13125_amd import binding as B
    from paper_2007_13125_amd.binding import Plan
    data = (to_dev(w.v), to_dev(w.f), to_dev(w.fder))
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    B.pint_sequential_solve(plan.h, *data, U)          # warm-up (code objects, caches)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        B.pint_sequential_solve(plan.h, *data, U)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    plan.close()
    del U
    torch.cuda.empty_cache()
    return {"ms": best * 1e3, "steps": w.N, "precision": "fp64"}


def bench_heat1d(args, refs):
    """The small 1D workload: launch-bound (4032 unknowns); sweeps/s and the time to a
    trajectory within 1e-12 of the oracle, FP64 residual form."""
    import torch

    from paper_2007_13125_amd import workloads as wl
    w = wl.heat1d()
    steps = max(args.steps, 50)
    plan, U, ms_ev, slots, var = run_variant(w, "fp64", "residual", steps, args.warmup, False)
    # the sweep rate without the per-launch event pairs of the profiled run (at this size
    # they are a sizeable part of a sweep): the same number of sweeps, launched back to back
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.sweeps(U, steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    e = {"workload": DESCR["heat1d"], "unknowns": w.N * w.M, "ms_per_step": ms, "sweeps_per_s": 1e3 / ms,
         "ms_per_step_with_launch_events": ms_ev, "kernels_ms": slot_summary(slots)}
    if refs is not None:
        e["time_to_1e-12"] = time_to_tol(plan, U, sampler(w)[1], refs["heat1d"], 1e-12, 20)
    plan.close()
    torch.cuda.synchronize()
    return e


def bench_batch(count=256):
    """The many-instance recipe (count instances, seed (4, i)), mixed precision, stop
    test 1e-10 on the update: all of its 1D instances in one pint_batch_solve (batched
    sweeps), beside the same instances solved one plan after another, and the four
    smallest 2D instances one plan each (the
    single-plan path that batches take for them, autotuned).  The 2D instances of the
    full recipe (up to 1023^2 x 1024 unknowns each, 1.3e10 in all) are not run here:
    their host-side data generation alone would take many minutes."""
    import torch

    from paper_2007_13125_amd import binding as B
    from paper_2007_13125_amd import workloads as wl
    params = [wl.batch_params(i) for i in range(count)]
    one = [i for i in range(count) if params[i][0] == 1]
    two = sorted([i for i in range(count) if params[i][0] == 2],
                 key=lambda i: params[i][2] * params[i][1][0] * params[i][1][1])[:4]
    ws = [wl.batch_instance(i) for i in one]
    S = 40
    grids = [B.make_grid(w.m) for w in ws]
    prm = [B.make_params(w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-10, max_sweeps=S, precision="mixed") for w in ws]
    h = B.pint_batch_plan_create(grids, prm)
    data = [(to_dev(w.v), to_dev(w.f), to_dev(w.fder)) for w in ws]
    Us = [torch.empty((w.N, w.M), dtype=torch.float64, device="cuda") for w in ws]
    args = ([d[0] for d in data], [d[1] for d in data], [d[2] for d in data], Us, S)
    B.pint_batch_solve(h, *args)                 # warm-up (code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, upd, sw = B.pint_batch_solve(h, *args)
    torch.cuda.synchronize()
    t1d = time.perf_counter() - t0
    B.pint_plan_destroy(h)
    # the same instances one plan after another (single-plan path, no tuning)
    plans = [B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-10, max_sweeps=S, precision="mixed") for w in ws]
    for p, d, U in zip(plans, data, Us):
        p.solve(*d, U=U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, d, U in zip(plans, data, Us):
        p.solve(*d, U=U)
    torch.cuda.synchronize()
    tone = time.perf_counter() - t0
    for p in plans:
        p.close()
    upd1 = sum(w.N * w.M * s for w, s in zip(ws, sw))
    out = {"recipe": f"{count} instances, seed (4, i), mixed, tol 1e-10", "n_1d": len(one),
           "unknowns_1d": sum(w.N * w.M for w in ws), "status_1d": st, "sweeps_1d_max": max(sw),
           "sweeps_1d_mean": float(sum(sw)) / len(sw), "ms_1d": t1d * 1e3,
           "unknown_updates_per_s_1d": upd1 / t1d, "ms_1d_one_plan_each": tone * 1e3}
    del Us, data
    torch.cuda.empty_cache()
    rows = []
    for i in two:
        w = wl.batch_instance(i)
        plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-10, max_sweeps=S, precision="mixed")
        plan.set_autotune(2)
        d = (to_dev(w.v), to_dev(w.f), to_dev(w.fder))
        plan.solve(*d)                            # warm-up + tuning
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, info = plan.solve(*d)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows.append({"instance": i, "grid": list(w.m), "N": w.N, "k": w.k, "alpha": w.alpha, "kappa": w.kappa,
                     "sweeps": info["sweeps"], "ms": dt * 1e3,
                     "unknown_updates_per_s": w.N * w.M * info["sweeps"] / dt})
        plan.close()
        del U, d
        torch.cuda.empty_cache()
    out["smallest_2d"] = rows
    return out


# ---------------------------------------------------------------------------------------
# CPU leg: the FP64 oracle (test infrastructure) timed on a bounded sample of the
# headline workload, and the oracle's values that time-to-tolerance is measured against

def wall_ms(fn, reps=3):
    """Median wall-clock time (ms) of fn() over reps runs after one warm-up run,
    each bracketed by device synchronisation (the solves run their host stop
    tests, so wall time is what a caller sees); returns (ms, last result)."""
    import torch
    out = fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return sorted(ts)[len(ts) // 2], out


def bench_next():
    """The rows beyond the single linear sweep, each at the paper's size and at a
    larger one: Algorithm 3 (Allen-Cahn, Sec. 4 Example 4), P1 elements (Example 1's
    problem with the paper's elements, against the same problem with finite
    differences) and windowed solves (2D heat in 4 windows against one solve)."""
    import torch
    from paper_2007_13125_amd import binding as B
    from paper_2007_13125_amd import workloads as wl
    out = {}
    rows = []
    for M, N in ((999, 100), (2047, 1024)):
        w, c3, c1 = wl.example4(2, 0.75, M=M, N=N)
        plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-12, max_sweeps=40)
        U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
        v, f, fd = to_dev(w.v), to_dev(w.f), to_dev(w.fder)
        ms, (st, inner, upd) = wall_ms(lambda: B.pint_nonlinear_solve(plan.h, c3, c1, v, f, fd, U, 3))
        plan.close()
        rows.append({"problem": f"Allen-Cahn, eps=1, kappa=0.1, T=0.4, m={M}, N={N}, BDF2, alpha=0.75, "
                                f"3 Newton steps (Table 4's protocol)",
                     "ms": ms, "inner_sweeps": inner, "max_update_per_newton_step": upd,
                     "unknown_updates_per_s": w.N * w.M * sum(inner) / (ms * 1e-3)})
    out["algorithm3"] = rows
    rows = []
    for label, wf, wd in (("Example 1 (Table 2's problem), m=999, N=100, BDF6", wl.example1_fem(6), wl.example1(6)),
                          ("1D heat line m=2047, N=2048, BDF2",
                           wl.fem1d(m=2047, N=2048, k=2), wl.heat1d(seed=61, m=2047, N=2048, k=2))):
        rec = {"problem": label}
        for space, w in (("fem", wf), ("fd", wd)):
            plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-12, max_sweeps=40, space=space)
            U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
            v, f, fd = to_dev(w.v), to_dev(w.f), to_dev(w.fder)
            ms, (_, info) = wall_ms(lambda: plan.solve(v, f, fd, U))
            plan.close()
            rec[space] = {"ms_to_1e-12": ms, "sweeps": info["sweeps"], "status": info["status"]}
        rows.append(rec)
    out["fem_p1"] = rows
    w = wl.heat2d(k=2)
    nwin = 4
    v, f = to_dev(w.v), to_dev(w.f)
    plan = B.Plan(w.m, w.k, w.alpha, w.T / nwin, w.N // nwin, w.kappa, tol=1e-12, max_sweeps=40)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device="cuda")
    ms_w, (st, _, sw) = wall_ms(lambda: B.pint_solve_windows(plan.h, nwin, v, f, None, U, 40))
    ws_w = B.pint_plan_workspace_bytes(plan.h)
    plan.close()
    plan = B.Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-12, max_sweeps=40)
    ms_1, (_, info) = wall_ms(lambda: plan.solve(v, f, None, U))
    ws_1 = B.pint_plan_workspace_bytes(plan.h)
    plan.close()
    out["windows"] = {"problem": "2D heat 255^2, N=512, BDF2, kappa=1e-5, tol 1e-12: 4 windows of 128 steps "
                                 "against one solve of 512",
                      "windows": {"ms": ms_w, "sweeps_per_window": sw, "status": st, "workspace_bytes": ws_w},
                      "one_solve": {"ms": ms_1, "sweeps": info["sweeps"], "workspace_bytes": ws_1}}
    torch.cuda.empty_cache()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def modal_reference(w, dofs):
    """The sequential oracle (O1) in sine-mode space for data that are finite sine
    series: each mode evolves by the scalar scheme with the sum of its axis
    eigenvalues; the trajectory is assembled at the sampled dofs."""
    import numpy as np
    import scipy.sparse as sp

    from oracle.grid import Grid, sine_eigenvalues
    from oracle.sequential import sequential
    from paper_2007_13125_amd.workloads import _cos_profile_derivs
    g = Grid(w.m)
    cv, cf = w.modes["v"], w.modes["f"]
    shape = cv.shape
    mus = [sine_eigenvalues(g.m[a], g.h[a])[:shape[a]] for a in range(g.dim)]
    mu = sum(np.meshgrid(*mus, indexing="ij")).reshape(-1)
    f, fder = _cos_profile_derivs(w.N, w.T, w.k, cf.reshape(-1))
    C = sequential(sp.diags(mu), w.k, w.alpha, w.T, w.N, cv.reshape(-1), f, fder)
    rem, coords = np.asarray(dofs), []
    for a in range(g.dim):
        coords.append(rem % g.m[a])
        rem = rem // g.m[a]
    phi = np.ones((C.shape[1], len(dofs)))
    idx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    for a in range(g.dim):
        phi *= np.sin(np.pi * np.outer(idx[a].reshape(-1) + 1, coords[a] + 1) / (g.m[a] + 1))
    return C @ phi


def subdiff_modal_reference(w):
    """O1 on the sampled sine modes of the subdiffusion workload, from the modes'
    coefficients of v (every mode of A_h evolves by the scalar scheme)."""
    import numpy as np
    import scipy.sparse as sp

    from oracle.grid import sine_eigenvalues
    from oracle.sequential import sequential
    mx, my = w.m
    sx = np.sin(np.pi * np.outer(np.arange(1, mx + 1), MODE_IDX + 1) / (mx + 1))
    sy = np.sin(np.pi * np.outer(np.arange(1, my + 1), MODE_IDX + 1) / (my + 1))
    cv = 4.0 / ((mx + 1) * (my + 1)) * (sx.T @ w.v.reshape(my, mx).T @ sy)
    mu = (sine_eigenvalues(mx, 1.0 / (mx + 1))[MODE_IDX][:, None]
          + sine_eigenvalues(my, 1.0 / (my + 1))[MODE_IDX][None, :]).reshape(-1)
    return sequential(sp.diags(mu), w.k, w.alpha, w.T, w.N, cv.reshape(-1), None, None)


def cpu_leg(workloads, seconds_hint=12.0):
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.grid import Grid, laplacian
    from oracle.sequential import sequential
    from oracle.sweep import Problem
    from paper_2007_13125_amd import workloads as wl
    refs = {}
    for name, w in workloads.items():
        if name == "subdiff2d":
            refs[name] = subdiff_modal_reference(w)
        elif name == "heat1d":
            refs[name] = sequential(laplacian(Grid(w.m)), w.k, w.alpha, w.T, w.N, w.v, w.f, w.fder)
        else:
            refs[name] = modal_reference(w, sampler_dofs(w))
    # timed sample of the headline recipe: 11^3 grid, same N, k, kappa
    s = wl.heat3d(m=(11, 11, 11))
    A = laplacian(Grid(s.m))
    t0 = time.perf_counter()
    sequential(A, s.k, s.alpha, s.T, s.N, s.v, s.f, s.fder)
    t_o1 = time.perf_counter() - t0
    prob = Problem(A, s.k, s.alpha, s.T, s.N, s.kappa, s.v, s.f, s.fder)
    U = np.tile(s.v, (s.N, 1))
    reps, t = 0, 0.0
    while t < seconds_hint and reps < 5:
        t0 = time.perf_counter()
        U, _ = prob.sweep(U, "residual")
        t += time.perf_counter() - t0
        reps += 1
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    base = {"value": s.N * s.M * reps / t, "unit": "unknown-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} residual sweep(s) of the dense-DFT oracle (Algorithm 1, all N frequencies, "
                      f"refined sparse LU per frequency) on the headline recipe at 11^3 interior nodes, N=256, "
                      f"BDF6, kappa=1e-6: {t:.1f} s; the sequential oracle's time to solution on the same "
                      f"sample {t_o1:.2f} s ({s.N * s.M / t_o1:.3g} unknowns/s)",
            "o1_seconds": t_o1, "o2_seconds_per_sweep": t / reps, "cpu_model": cpu_model(),
            "logical_cpus": os.cpu_count()}
    return base, refs


def sampler_dofs(w):
    import numpy as np
    return np.random.default_rng(0).choice(w.M, 4096, replace=False)


# ---------------------------------------------------------------------------------------
# profile summaries (rocprofv3 CSV -> profiles/<workload>_{kernels.md,traffic.json})

def slot_of(kernel, dim):
    # the forward pass is one kernel, or the split pair k_resid + k_tfft
    if "k_inject" in kernel:
        return "direct_rhs_spectrum"
    if "k_fwd_" in kernel or "k_resid" in kernel or "k_tfft" in kernel:
        return "forward_cq_rhs_tfft" if "k_fwd_cq" in kernel else "forward_rhs_tfft"
    if "k_dst_rows" in kernel:
        return "dst_x"
    if "k_dst_cols" in kernel:
        return ("dst_y_solve" if dim == 2 else None)
    if "k_inv" in kernel:
        return "inverse_tfft_update"
    return None


def summarize(outdir, name):
    """Write the committed profile summary (markdown) and the HBM traffic record of
    one workload from rocprofv3 CSV output of the three runs listed in the summary:
    <outdir>/trace (--kernel-trace --stats), <outdir>/FETCH_SIZE, <outdir>/WRITE_SIZE
    (--pmc), each of `bench.py --only <name> --steps 5 --warmup 1 --no-cpu-baseline
    --copy-calibration --no-tune` (the built-in kernel variants, so that each pass
    launches one kernel)."""
    import csv
    from collections import defaultdict

    from paper_2007_13125_amd import workloads as wl
    w = getattr(wl, name)()

    def rows(sub, suffix):
        paths = glob.glob(os.path.join(outdir, sub, "**", "*" + suffix), recursive=True)
        if not paths:
            raise SystemExit(f"no *{suffix} under {os.path.join(outdir, sub)}")
        return list(csv.DictReader(open(paths[0])))

    def short(k):
        for pre in ("void ", "pint::", "(anonymous namespace)::"):
            k = k.replace(pre, "")
        return k.split("(")[0]

    stats = rows("trace", "kernel_stats.csv")
    counters = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        per = defaultdict(list)
        for r in rows(c, "counter_collection.csv"):
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        counters[c] = per
    copies = [k for k in counters["FETCH_SIZE"] if "copyBuffer" in k or "copy" in k.lower()]
    fcal = max(max(counters["FETCH_SIZE"][k]) for k in copies)
    wcal = max(max(counters["WRITE_SIZE"][k]) for k in copies)
    rf, wf = COPY_BYTES / (fcal * 1024), COPY_BYTES / (wcal * 1024)
    sha = sources_sha()
    rec = {"workload": DESCR[name], "sources": KERNEL_SOURCES, "sources_sha256": sha, "variants": [0, 0, 0, 0],
           "calibration": {"copy_bytes": COPY_BYTES, "FETCH_SIZE_KiB": fcal, "WRITE_SIZE_KiB": wcal,
                           "read_factor": rf, "write_factor": wf},
           "kernels": {"fp64": {}, "mixed": {}}}
    stem = profile_stem(w)
    lines = [f"# Kernel profile: {DESCR[name]}", "",
             f"Device: one MI355X (gfx950).  Kernel sources sha256 prefix `{sha[:16]}`.", "",
             "Commands (run from /tmp with TMPDIR=/tmp; each writes CSV under the -d folder), then "
             f"`python bench.py --summarize <out> --only {name}` writes this file and the traffic record:", "",
             "```"]
    cmd = (f"python3 /root/repo/bench.py --only {name} --steps 5 --warmup 1 --no-cpu-baseline --copy-calibration "
           f"--no-tune")
    lines += [f"rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o {name} -- {cmd}",
              f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/FETCH_SIZE -o {name} -- {cmd}",
              f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/WRITE_SIZE -o {name} -- {cmd}",
              "```", "",
              "bench.py runs the FP64 plan (kernels `<double,...>`), the mixed plan (`<float,...>`) and the FP64 "
              "direct-form plan with the built-in kernel variants, each for its warmup and timed sweeps.", "",
              "## --kernel-trace --stats", "",
              "| kernel | calls | average us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{short(r['Name'])[:100]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", "## --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch, mean over dispatches)", "",
              f"Calibration: a plain {COPY_BYTES >> 20} MiB device copy read FETCH_SIZE = {fcal:.0f} KiB and "
              f"WRITE_SIZE = {wcal:.0f} KiB, so HBM read bytes = {rf:.3f} x FETCH_SIZE KiB x 1024 and write "
              f"bytes = {wf:.3f} x WRITE_SIZE KiB x 1024.", "",
              "", 
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB |",
              "|---|---|---|---|---|---|"]
    # per (precision, pass): the kernel with the most dispatches, or the split
    # forward pair (launched once each per sweep, traffic summed)
    parts = {}
    for k, vals in counters["FETCH_SIZE"].items():
        fk = sum(vals) / len(vals)
        wv = counters["WRITE_SIZE"].get(k, [0.0])
        wk = sum(wv) / len(wv)
        rd, wr = rf * fk * 1024, wf * wk * 1024
        lines.append(f"| `{short(k)[:100]}` | {len(vals)} | {fk:.4g} | {wk:.4g} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
        slot = slot_of(k, w.dim)
        if slot is None:
            continue
        prec = "mixed" if "<float" in k else "fp64"
        parts.setdefault((prec, slot), []).append((len(vals), rd, wr, short(k)))
    for (prec, slot), ks in parts.items():
        n = max(x[0] for x in ks)
        top = [x for x in ks if x[0] == n]
        pair = [x for x in top if x[3].startswith(("k_resid", "k_tfft"))]
        # the split pair is one pass; otherwise the first kernel of the pass (the
        # residual-form plan runs before the direct-form one)
        sel = pair if len(pair) == 2 else top[:1]
        rec["kernels"][prec][slot] = {"read": sum(x[1] for x in sel), "write": sum(x[2] for x in sel),
                                      "kernel": " + ".join(x[3] for x in sel), "dispatches": n}
    open(stem + "_kernels.md", "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(stem + "_traffic.json", "w"), indent=1)
    print(f"wrote {stem}_kernels.md and _traffic.json")


# ---------------------------------------------------------------------------------------

def main():
    global MODE_IDX
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (and with it the time-to-tolerance figures)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in kernel variants (no autotuning)")
    ap.add_argument("--only", choices=SWEEP_WORKLOADS + ("heat1d",),
                    help="run one workload only (profiling runs); it becomes the reported line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 256 MiB on the device (counter calibration for profiles)")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write the profile summary of --only's workload from rocprofv3 CSV in DIR and exit")
    args = ap.parse_args()
    import numpy as np
    MODE_IDX = np.array([0, 1, 2, 3, 4, 6, 9, 14, 22, 35, 56, 90, 145, 233, 376, 510])
    if args.summarize:
        summarize(args.summarize, args.only or HEADLINE)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs a sweep on one "
              f"GPU; sharding the dofs for the time FFTs and the frequencies for the spatial solves over several "
              f"GPUs is a design, not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2007_13125_amd import workloads as wl
    names = [args.only] if args.only else list(SWEEP_WORKLOADS) + ["heat1d"]
    ws = {n: getattr(wl, n)() for n in names}
    base, refs = (None, None)
    if not args.no_cpu_baseline:
        print("[bench] cpu leg", file=sys.stderr, flush=True)
        base, refs = cpu_leg(ws)
    results = {}
    for n in names:
        results[n] = bench_heat1d(args, refs) if n == "heat1d" else bench_workload(ws[n], args, refs)
        torch.cuda.empty_cache()
    head = args.only or HEADLINE
    h = results[head]
    w = ws[head]
    if head == "heat1d":
        res = {"metric": METRIC, "value": w.N * w.M / (h["ms_per_step"] * 1e-3), "ms_per_step": h["ms_per_step"]}
    else:
        res = {"metric": METRIC, "value": h["fp64"]["value"], "ms_per_step": h["fp64"]["ms_per_step"]}
    res.update({
        "unit": "unknown-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{head}: {DESCR[head]}, residual form, FP64 (mixed FP32/FP64 and the FP64 "
                               f"direct form alongside)", "grid": list(w.m), "N": w.N, "k": w.k,
                   "alpha": w.alpha, "kappa": w.kappa, "unknowns": w.N * w.M},
    })
    if head != "heat1d":
        res["roofline"] = h["fp64"]["roofline"]
        res["mixed"] = h["mixed"]
        res["fp64_direct"] = h["fp64_direct"]
        res["fp64"] = h["fp64"]
        if "sequential" in h:
            res["sequential"] = h["sequential"]
    if base is not None:
        res["cpu_baseline"] = base
    res["workloads"] = {n: r for n, r in results.items() if n != head}
    if not args.only:
        print("[bench] batch", file=sys.stderr, flush=True)
        res["workloads"]["batch"] = bench_batch()
        print("[bench] algorithm 3, P1 elements, windows", file=sys.stderr, flush=True)
        res["workloads"]["next_rows"] = bench_next()
    res["variant_knobs"] = ["forward kernel", "x pass rows", "y/z pass columns", "1D solver"]
    print(json.dumps(res), flush=True)
    if args.copy_calibration:
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
