"""Benchmark of the diagonalized waveform-relaxation sweep on one MI355X.

One step = one whole WR sweep (residual + kappa scaling + forward time FFT,
spatial shifted solves, inverse time FFT + unscale + update + norms) over the
2D heat workload: 5-point FD Laplacian on 255 x 255 interior nodes, BDF4,
T = 1, N = 512, kappa = 1e-5, seeded smooth sine-series data.  Inputs are
resident in HBM before the timed region.

Prints ONE JSON line with the FP64 sweep throughput (space-time unknown
updates per second) as `value`, the mixed FP32/FP64 sweep alongside,
per-kernel device times from HIP events recorded on the plan's stream inside
the timed region, the HBM roofline of the dominant kernel, time-to-1e-10 for
both precisions, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "space-time unknown-updates/s per WR sweep + time-to-1e-10, FP64 vs mixed; %HBM"
HBM_PEAK_GBS = 8000.0


def spectrum_bytes(N, M, mixed):
    return (N // 2 + 1) * M * (8 if mixed else 16)


def kernel_bytes(name, N, M, mixed, has_f):
    """Algorithmic HBM bytes of one launch (each array read or written once)."""
    S = spectrum_bytes(N, M, mixed)
    if name.startswith("forward"):
        return 8 * N * M + (8 * N * M if has_f else 0) + 8 * M + S   # U, f, v in; spectrum out
    if name.startswith("inverse"):
        return S + 16 * N * M                                       # spectrum in; U in and out
    if name == "norm_reduce":
        return 0
    return 2 * S                                                    # spatial pass: spectrum in and out


def measured_traffic(precision, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record, or None when the kernel source changed since it was taken."""
    import hashlib
    rec_path = PROFILE_STEM + "_traffic.json"
    try:
        rec = json.load(open(rec_path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        k = rec["kernels"][precision][kernel]
        return k["read"] + k["write"]
    except (OSError, KeyError, ValueError):
        return None


def run_precision(w, precision, steps, warmup, form="residual", tune=True):
    import torch

    from paper_2007_13125_amd.binding import Plan
    dev = torch.device("cuda")
    v = torch.from_numpy(w.v).to(dev)
    f = torch.from_numpy(w.f).to(dev) if w.f is not None else None
    fd = torch.from_numpy(w.fder).to(dev) if w.fder is not None else None
    plan = Plan(w.m, w.k, w.alpha, w.T, w.N, w.kappa, tol=1e-14, max_sweeps=30, precision=precision, form=form)
    plan.bind(v, f, fd)
    U = torch.empty((w.N, w.M), dtype=torch.float64, device=dev)
    plan.init_iterate(U)
    # kernel variants chosen by the library's autotuner (plan setup, outside the timed region)
    variants = plan.tune(U, 3) if tune else plan.variants()
    plan.init_iterate(U)
    if warmup:
        plan.sweeps(U, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prof = plan.profile(U, steps)          # the timed region: HIP events around every launch
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) / steps * 1e3
    return plan, (v, f, fd), ms_per_step, prof, variants


def time_to_tol(w, plan, data, Uref, tol=1e-10, max_sweeps=12):
    """Sweeps m* until the trajectory is within tol (relative L2) of Uref, found in an
    untimed validation run; then the wall time of exactly m* sweeps from U_0."""
    import torch
    U = torch.empty_like(Uref)
    plan.init_iterate(U)
    nref = torch.linalg.norm(Uref).item()
    mstar, errs = None, []
    for s in range(1, max_sweeps + 1):
        plan.sweeps(U, 1)
        e = (torch.linalg.norm(U - Uref).item()) / nref
        errs.append(e)
        if e <= tol:
            mstar = s
            break
    if mstar is None:
        return {"sweeps": None, "ms": None, "errors": errs}
    best = float("inf")
    for _ in range(3):
        plan.init_iterate(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.sweeps(U, mstar)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return {"sweeps": mstar, "ms": best * 1e3, "errors": errs}


def other_configs(steps, tune):
    """The other multi-dimensional workloads of the method's evaluation (parity-test
    cases, not bench lines): tuned sweep time per precision and its algorithmic
    HBM fraction."""
    import torch

    from paper_2007_13125_amd import workloads as wl
    out = {}
    for name in ("subdiff2d", "heat3d"):
        w = getattr(wl, name)()
        entry = {"grid": list(w.m), "N": w.N, "k": w.k, "alpha": w.alpha, "kappa": w.kappa, "unknowns": w.N * w.M}
        for precision in ("fp64", "mixed"):
            plan, _, ms, prof, var = run_precision(w, precision, steps, 1, tune=tune)
            mixed = precision == "mixed"
            nbytes = sum(kernel_bytes(n, w.N, w.M, mixed, w.f is not None) for n, _ in prof)
            entry[precision] = {"ms_per_step": ms, "value": w.N * w.M / (ms * 1e-3),
                                "sweep_hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "kernels_ms": {n: t for n, t in prof}, "variants": var}
            plan.close()
            torch.cuda.empty_cache()
        out[name] = entry
    return out


def cpu_baseline(seconds_hint=20.0):
    """The FP64 oracle's dense-DFT sweep (Algorithm 1 with dense DFT matrices and
    sparse LU per frequency), timed on a bounded sample: the same recipe on a
    63 x 63 grid with the same N = 512 and BDF4."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.grid import Grid, laplacian
    from oracle.sweep import Problem
    from paper_2007_13125_amd import workloads as wl
    w = wl.heat2d(m=(63, 63))
    prob = Problem(laplacian(Grid(w.m)), w.k, w.alpha, w.T, w.N, w.kappa, w.v, w.f, w.fder)
    U = np.tile(w.v, (w.N, 1))
    reps, t = 0, 0.0
    while t < seconds_hint and reps < 5:
        t0 = time.perf_counter()
        U, _ = prob.sweep(U, "residual")
        t += time.perf_counter() - t0
        reps += 1
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": w.N * w.M * reps / t, "unit": "unknown-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} residual sweep(s) of the dense-DFT oracle on the 63x63 grid, N=512, BDF4 "
                      f"(same recipe as the timed workload); {t:.1f} s; host logical CPUs {os.cpu_count()}"}


PROFILE_STEM = os.path.join(ROOT, "profiles", "heat2d_255x255_N512_bdf4")
KERNEL_SOURCE = "paper_2007_13125_amd/csrc/pint_kernels.hip"
COPY_BYTES = 256 << 20


def slot_of(kernel):
    """Profile slot of a kernel symbol of the 2D sweep (bench workload)."""
    if "k_fwd_" in kernel:
        return "forward_rhs_tfft"
    if "k_dst_rows" in kernel:
        return "dst_x"
    if "k_dst_cols" in kernel:
        return "dst_y_solve"
    if "k_inv" in kernel:
        return "inverse_tfft_update"
    return None


def summarize(outdir):
    """Write the committed profile summary (markdown) and the HBM traffic record
    that bench.py reads, from rocprofv3 CSV output of the three runs listed in
    the summary: <outdir>/trace (--kernel-trace --stats), <outdir>/FETCH_SIZE and
    <outdir>/WRITE_SIZE (--pmc), each of `bench.py --steps 5 --warmup 1
    --no-cpu-baseline --copy-calibration`."""
    import csv
    import glob
    import hashlib
    from collections import defaultdict

    def rows(sub, suffix):
        paths = glob.glob(os.path.join(outdir, sub, "**", "*" + suffix), recursive=True)
        if not paths:
            raise SystemExit(f"no *{suffix} under {os.path.join(outdir, sub)}")
        return list(csv.DictReader(open(paths[0])))

    def short(name):
        for pre in ("void ", "pint::", "(anonymous namespace)::"):
            name = name.replace(pre, "")
        return name.split("(")[0]

    stats = rows("trace", "kernel_stats.csv")
    counters = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        per = defaultdict(list)
        for r in rows(c, "counter_collection.csv"):
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        counters[c] = per
    # calibration: the largest device copy (the 256 MiB copy of --copy-calibration)
    copies = [k for k in counters["FETCH_SIZE"] if "copyBuffer" in k]
    fcal = max(max(counters["FETCH_SIZE"][k]) for k in copies)
    wcal = max(max(counters["WRITE_SIZE"][k]) for k in copies)
    rf, wf = COPY_BYTES / (fcal * 1024), COPY_BYTES / (wcal * 1024)
    src = open(os.path.join(ROOT, KERNEL_SOURCE), "rb").read()
    sha = hashlib.sha256(src).hexdigest()
    rec = {"workload": "heat2d 255x255 N=512 BDF4 kappa=1e-5", "source": KERNEL_SOURCE, "source_sha256": sha,
           "calibration": {"copy_bytes": COPY_BYTES, "FETCH_SIZE_KiB": fcal, "WRITE_SIZE_KiB": wcal,
                           "read_factor": rf, "write_factor": wf},
           "kernels": {"fp64": {}, "mixed": {}}}
    lines = ["# Kernel profile: 2D heat 255x255, N=512, BDF4, kappa=1e-5 (bench workload)", "",
             f"Device: one MI355X (gfx950).  Source: `{KERNEL_SOURCE}` sha256 prefix `{sha[:16]}`.", "",
             "Commands (run from /tmp with TMPDIR=/tmp; each writes CSV under the -d folder), then "
             "`python bench.py --summarize <out>` writes this file and the traffic record:", "", "```"]
    cmd = "python3 /root/repo/bench.py --steps 5 --warmup 1 --no-cpu-baseline --no-other-configs --copy-calibration"
    lines += [f"rocprofv3 --kernel-trace --stats --output-format csv -d <out>/trace -o heat2d -- {cmd}",
              f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out>/FETCH_SIZE -o heat2d -- {cmd}",
              f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out>/WRITE_SIZE -o heat2d -- {cmd}",
              "```", "",
              "bench.py runs the FP64 plan (kernels `<double,...>`) and the mixed plan (`<float,...>`), each for "
              "warmup + timed + time-to-1e-10 sweeps.", "", "## --kernel-trace --stats", "",
              "| kernel | calls | average us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{short(r['Name'])[:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", "## --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch, mean over dispatches)", "",
              f"Calibration: a plain {COPY_BYTES >> 20} MiB device copy read FETCH_SIZE = {fcal:.0f} KiB and "
              f"WRITE_SIZE = {wcal:.0f} KiB, so HBM read bytes = {rf:.3f} x FETCH_SIZE KiB x 1024 and write "
              f"bytes = {wf:.3f} x WRITE_SIZE KiB x 1024.", "",
              "Kernels with few dispatches are the autotuner's trial launches of the variants not chosen.", "",
              "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | write MB |", "|---|---|---|---|---|"]
    # the autotuner also launches the other variants of a slot a few times: the
    # record keeps, per slot, the kernel with the most dispatches (the timed one)
    calls = {}
    for k, vals in counters["FETCH_SIZE"].items():
        slot = slot_of(k)
        if slot is None:
            continue
        fk = sum(vals) / len(vals)
        wk = sum(counters["WRITE_SIZE"][k]) / len(counters["WRITE_SIZE"][k])
        rd, wr = rf * fk * 1024, wf * wk * 1024
        prec = "mixed" if "<float" in k else "fp64"
        if len(vals) > calls.get((prec, slot), 0):
            calls[(prec, slot)] = len(vals)
            rec["kernels"][prec][slot] = {"read": rd, "write": wr, "kernel": short(k), "dispatches": len(vals)}
        lines.append(f"| `{short(k)}` | {fk:.4g} | {wk:.4g} | {rd / 1e6:.1f} | {wr / 1e6:.1f} |")
    open(PROFILE_STEM + "_kernels.md", "w").write("\n".join(lines) + "\n")
    json.dump(rec, open(PROFILE_STEM + "_traffic.json", "w"), indent=1)
    print(f"wrote {PROFILE_STEM}_kernels.md and _traffic.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in kernel variants (no autotuning)")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the sweep timings of the 2D subdiffusion and 3D heat workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 256 MiB on the device (counter calibration for profiles)")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write the profile summary from rocprofv3 CSV output in DIR and exit (no GPU)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args.summarize)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sharded multi-GPU "
              f"design is described in DESIGN.md and is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2007_13125_amd import workloads as wl
    w = wl.heat2d()
    N, M = w.N, w.M
    has_f = w.f is not None
    out = {}
    plans = {}
    for precision in ("fp64", "mixed"):
        plan, data, ms, prof, var = run_precision(w, precision, args.steps, args.warmup, tune=not args.no_tune)
        mixed = precision == "mixed"
        kern = {name: ms_k for name, ms_k in prof}
        sweep_bytes = sum(kernel_bytes(n, N, M, mixed, has_f) for n, _ in prof)
        dom = max(prof, key=lambda t: t[1])
        dom_bytes = kernel_bytes(dom[0], N, M, mixed, has_f)
        achieved = dom_bytes / (dom[1] * 1e-3) / 1e9
        out[precision] = {
            "value": N * M / (ms * 1e-3), "ms_per_step": ms, "kernels_ms": kern,
            "sweep_alg_bytes": sweep_bytes,
            "sweep_hbm_frac": sweep_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "dominant": {"kernel": dom[0], "ms": dom[1], "bytes": dom_bytes, "GBps": achieved},
            "variants": var,
        }
        plans[precision] = (plan, data)
    # reference trajectory for time-to-1e-10: the FP64 path converged to 1e-14
    # (the FP64 path matches the CPU oracle to ~1e-14 at this size in the parity tests)
    plan64, data64 = plans["fp64"]
    Uref = torch.empty((N, M), dtype=torch.float64, device="cuda")
    plan64.init_iterate(Uref)
    plan64.sweeps(Uref, 8)
    torch.cuda.synchronize()
    # the paper's direct form in FP64 (its roundoff floor, ~eps/kappa ~ 6e-12 here, is below 1e-10)
    pd, dd, ms_d, prof_d, var_d = run_precision(w, "fp64", args.steps, args.warmup, form="direct",
                                                tune=not args.no_tune)
    plans["fp64_direct"] = (pd, dd)
    ttt = {p: time_to_tol(w, plans[p][0], plans[p][1], Uref) for p in ("fp64", "fp64_direct", "mixed")}

    d = out["fp64"]["dominant"]
    res = {
        "metric": METRIC,
        "value": out["fp64"]["value"],
        "unit": "unknown-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": out["fp64"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "heat2d: 2D heat, 5-point FD Dirichlet Laplacian 255x255, BDF4 (Table 1 "
                               "corrections), T=1, N=512, kappa=1e-5, residual form, FP64",
                   "grid": list(w.m), "N": N, "k": w.k, "kappa": w.kappa, "form": "residual",
                   "unknowns": N * M},
        "roofline": {"bound": "hbm", "kernel": d["kernel"], "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["GBps"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic("fp64", d["kernel"]), "alg_bytes": d["bytes"]},
        "kernels_ms": out["fp64"]["kernels_ms"],
        "sweep_hbm_frac": out["fp64"]["sweep_hbm_frac"],
        "variants": {"fp64": out["fp64"]["variants"], "mixed": out["mixed"]["variants"], "fp64_direct": var_d,
                     "knobs": ["forward kernel", "x pass rows", "y pass columns", "1D tridiagonal split"]},
        "mixed": {k: out["mixed"][k] for k in ("value", "ms_per_step", "kernels_ms", "sweep_hbm_frac",
                                               "dominant")},
        # relative L2 error after each sweep (against the FP64 path converged to ~1e-14)
        "time_to_1e-10": {p: {"sweeps": ttt[p]["sweeps"], "ms": ttt[p]["ms"],
                              "rel_l2_per_sweep": [float("%.3g" % e) for e in ttt[p]["errors"]]} for p in ttt},
        "fp64_direct": {"ms_per_step": ms_d, "kernels_ms": {n: t for n, t in prof_d}},
    }
    if not args.no_other_configs:
        res["other_configs"] = other_configs(5, not args.no_tune)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline()
    for p in plans.values():
        p[0].close()
    print(json.dumps(res), flush=True)
    if args.copy_calibration:
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
