"""Benchmark: all-omega time-to-solution of the split Krylov solver on one GPU.

A step is one full solve of the 128^3 plain-method workload (12.6M unknowns,
2000 random spheres, 8-cell quadratic absorbing layer, omega = 2 pi 0.1,
T = 500, Krylov dimension 64, tol 1e-8): shifted solve for z, transient
e^{-TA} Im z by restarts in time, and the split assembly.  Inputs (materials
and the source) are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is the time to solution in seconds (lower is
better); the roofline object reports the dominant kernel's achieved HBM
bandwidth from per-launch HIP events recorded on the solver's stream during
the timed steps, against MI355X's 8 TB/s; cpu_baseline is the FP64 oracle
timed on the host on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_128cube_traffic.md")
# kernel class -> (kernel in the counter summary, source file it is built from)
CLASS_KERNEL = {"block_gram": ("k_gram_step_lds", "kry_block.hip"),
                "block_gemm": ("k_gemm_cols", "kry_block.hip"),
                "operator": ("k_stencil_axpby", "kry_kernels.hip")}


def measured_traffic(kernel_class, workload, alg_bytes_per_launch):
    """HBM bytes per launch of the class's kernel: the ratio of counted to
    algorithmic bytes from the committed counter summary (two rocprofv3
    --pmc runs of this script with --calibration-copy) times this run's
    algorithmic bytes per launch; None if there is no summary or the kernel
    source changed since."""
    import hashlib
    import re
    if workload != "c2" or kernel_class not in CLASS_KERNEL or not os.path.exists(TRAFFIC_FILE):
        return None
    kernel, source = CLASS_KERNEL[kernel_class]
    src = os.path.join(ROOT, "paper_1707_00023_amd", "csrc", source)
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    pat = re.compile(r"traffic_ratio (\S+) (\S+) source_sha256_16 (\S+)")
    for line in open(TRAFFIC_FILE):
        m = pat.search(line)
        if m and m.group(1) == kernel and m.group(3) == h:
            return float(m.group(2)) * alg_bytes_per_launch
    return None


def host_info():
    """The host the CPU baseline ran on: usable CPUs, CPU model, memory."""
    info = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
            else os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_gb"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def cpu_baseline(wl, inp):
    """The oracle's y(T) for the workload's column, timed on this host.

    The oracle route is the augmented-matrix exponential action (one
    expm_multiply of the (n + 2) system; no shifted solve).  A full run at
    T = 500 takes 10-50 minutes, so two short horizons are timed and the
    cost is extrapolated linearly in T (a fixed norm-estimation part plus a
    per-time-unit part).  The model was checked at full size on one host:
    horizons 5, 10, 20 extrapolate to 2984 s where the full run took 2762 s.
    Threads are not restricted; SciPy's sparse products run on one core, so
    the effective core count (process CPU time over wall time) is reported."""
    import workloads as wk
    from oracle import operator as op
    from oracle import solve as osv

    A = op.assemble_A(inp.eps, inp.mu, inp.sigma)
    b = wk.source_vector(wl, wl.omegas[0], 0.0)
    T1, T2 = wl.T / 100.0, wl.T / 50.0
    times, cpu = [], 0.0
    for Ts in (T1, T2):
        c0, t0 = time.process_time(), time.perf_counter()
        osv.augmented_solution(A, b, wl.omegas[0], Ts)
        times.append(time.perf_counter() - t0)
        cpu += time.process_time() - c0
    slope = (times[1] - times[0]) / (T2 - T1)
    est = times[0] + slope * (wl.T - T1)
    eff = cpu / sum(times)
    return {"value": est * len(wl.omegas), "unit": "s", "cores": max(1, int(round(eff))),
            "kind": "oracle", "extrapolated": True,
            "effective_cores": round(eff, 2), "host": host_info(),
            "sample": (f"oracle augmented-matrix expm_multiply for one column timed at "
                       f"t={T1:g} and t={T2:g} ({times[0]:.1f}s, {times[1]:.1f}s wall), "
                       f"extrapolated linearly to T={wl.T:g} and all {len(wl.omegas)} omega")}


FP64_MFMA_PEAK_TFLOPS = 78.6


def _kernel_entry(st, i):
    """Per-class totals of one solve: time, launches, GB/s and (matrix-core
    classes) TFLOP/s against the FP64 matrix peak."""
    ms = st["kernel_ms"][i]
    e = {"ms": ms, "launches": st["kernel_launches"][i],
         "gbs": st["kernel_bytes"][i] / (ms * 1e6) if ms > 0 else 0.0}
    if st["kernel_flops"][i] > 0 and ms > 0:
        tf = st["kernel_flops"][i] / (ms * 1e9)
        e["tflops"] = tf
        e["mfma_frac"] = tf / FP64_MFMA_PEAK_TFLOPS
    return e


def compare_batched(args, wl, inp, dev):
    """Batched multi-omega solves against plain per-column solves of the same
    columns at the same tolerance: `columns` consecutive frequencies of the
    workload at one incidence angle (per-frequency oblique sources).
    plain: every column on its own; continuation: the columns solved in
    frequency order, each shifted solve starting from the extrapolation of
    the earlier frequencies' solutions (continuation_transient: the
    transients continued too, equation (4diff)); block: the columns sharing
    one block Krylov space (block width, block steps); restarted: the
    residual-restarted method with every column's source expressed in one
    shared real basis, whose sequences of bases serve all columns.
    --theta-index -1 takes every angle of each frequency (columns = the
    frequencies times the angles)."""
    import numpy as np
    import torch

    import paper_1707_00023_amd as kry
    import workloads as wk

    eps = torch.as_tensor(inp.eps, device=dev)
    sig = torch.as_tensor(inp.sigma, device=dev)
    ks = list(range(args.omega_index, min(args.omega_index + args.columns, len(wl.omegas))))
    om = [wl.omegas[k] for k in ks]
    # one source per (frequency, angle): column (k, s) at k * n_angles + s
    angles = [float(t) for t in inp.thetas] if args.theta_index < 0 else [float(inp.thetas[args.theta_index])]
    th = angles[0] if args.theta_index >= 0 else "all"
    B = torch.as_tensor(np.stack([wk.source_vector(wl, w, t) for w in om for t in angles]), device=dev)
    out = {"metric": "batched vs plain time to solution (same columns, same tol)",
           "workload": wl.name, "columns": B.shape[0], "omegas": om, "theta": th, "T": wl.T,
           "tol": wl.tol}
    ys = {}
    all_modes = {"plain": {}, "continuation": {"omega_continuation": True},
                 "continuation_transient": {"omega_continuation": True, "transient_continuation": True},
                 "block": {"block_width": args.block_width, "block_steps": args.block_steps},
                 "restarted": {}}
    names = ([] if args.skip_plain else ["plain"]) + [m for m in args.batched_modes.split(",")
                                                        if m in all_modes and m != "plain"]
    modes = [(m, all_modes[m]) for m in names]
    for name, extra in modes:
        s = kry.Solver(eps, None, sig, kry.Options(krylov_dim=wl.krylov_dim, tol=wl.tol, timing=True,
                                                   s_step=args.s_step, verbose=args.verbose,
                                                   **extra))
        solve = s.solve_restarted if name == "restarted" else s.solve_multifreq
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = solve(om, B, wl.T, b_per_omega=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = s.last_stats
        ys[name] = y.cpu().numpy()
        out[name] = {"s": dt, "s_per_column": dt / B.shape[0],
                     "stationary_s": st["ms_stationary"] / 1e3, "transient_s": st["ms_transient"] / 1e3,
                     "matvecs_stationary": st["matvecs_stationary"],
                     "matvecs_transient": st["matvecs_transient"],
                     "max_residual": st["max_residual"],
                     "kernels": {k: _kernel_entry(st, i) for i, k in enumerate(kry.KERNEL_CLASSES)
                                 if st["kernel_launches"][i] > 0}}
        print(f"[bench] {name}: {dt:.1f} s", file=sys.stderr, flush=True)
        s.close()
    for name in names:
        if name == "plain" or "plain" not in ys:
            continue
        d = np.linalg.norm(ys[name] - ys["plain"], axis=1) / np.linalg.norm(ys["plain"], axis=1)
        out[name]["max_rel_diff_vs_plain"] = float(d.max())
        out[name]["speedup_vs_plain"] = out["plain"]["s"] / out[name]["s"]
    if wl.name.startswith("c3") and args.golden_check:
        # the stored oracle columns that fall among the solved ones
        g = json.load(open(os.path.join(ROOT, "tests", "golden", "c3_yT_samples.json")))
        idx = np.asarray(g["indices"])
        checks = []
        for col in g["columns"]:
            if col["omega_index"] not in ks or (args.theta_index >= 0 and col["theta_index"] != args.theta_index):
                continue
            k = ks.index(col["omega_index"]) * len(angles) + (col["theta_index"] if args.theta_index < 0 else 0)
            for name in names:
                yv = ys[name][k]
                checks.append({"mode": name, "omega_index": col["omega_index"], "theta_index": col["theta_index"],
                               "sampled_rel_err": float(np.linalg.norm(yv[idx] - np.asarray(col["values"]))
                                                        / np.linalg.norm(col["values"]))})
        out["oracle_columns"] = checks
    print(json.dumps(out), flush=True)


COPY_BYTES = 1 << 30


def precision_runs(wl, inp, dev, om, method, s_step, verbose=True):
    """All frequencies om of the workload's shared source, solved once with
    FP32 storage (FP32 stencil, FP64 reductions and small dense) at the
    workload's tolerance and once in FP64 at 1e-8, by the split solver
    (Corollary 3) or the residual-restarted method; wall time of each solve
    and the relative 2-norm error of every FP32 field against the FP64 one.
    Returns (summary dict, solutions by name)."""
    import torch

    import paper_1707_00023_amd as kry
    import workloads as wk

    eps = torch.as_tensor(inp.eps, device=dev)
    sig = torch.as_tensor(inp.sigma, device=dev)
    b = torch.as_tensor(wk.source_vector(wl, om[0], 0.0)[None, :], device=dev)
    out = {"metric": "FP32-storage error vs FP64 GPU run, per omega", "workload": wl.name,
           "n": wl.n, "omegas": om, "T": wl.T, "krylov_dim": wl.krylov_dim, "method": method}
    ys = {}
    for name, storage, tol in (("f32", "f32", wl.tol), ("f64", "f64", 1e-8)):
        s = kry.Solver(eps, None, sig, kry.Options(storage=storage, krylov_dim=wl.krylov_dim,
                                                   tol=tol, verbose=verbose, s_step=s_step))
        solve = s.solve_restarted if method == "restarted" else s.solve_multifreq
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = solve(om, b, wl.T)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = s.last_stats
        ys[name] = y
        out[name] = {"tol": tol, "s": dt, "matvecs_stationary": st["matvecs_stationary"],
                     "matvecs_transient": st["matvecs_transient"], "converged": bool(st["converged"]),
                     "gcell_updates_per_s": wl.N ** 3 * (st["matvecs_stationary"] + st["matvecs_transient"]) / dt / 1e9}
        print(f"[bench] {name}: {dt:.1f} s", file=sys.stderr, flush=True)
        s.close()
    err = (torch.linalg.norm(ys["f32"] - ys["f64"], dim=1) / torch.linalg.norm(ys["f64"], dim=1))
    out["rel_err_per_omega"] = [float(e) for e in err.cpu()]
    out["speedup_f32_over_f64"] = out["f64"]["s"] / out["f32"]["s"]
    return out, ys


def precision_compare(args, wl, inp, dev):
    """FP32 storage against an FP64 run of the same frequencies (see
    precision_runs), optionally checked against one-at-a-time FP64 solves."""
    import torch

    import paper_1707_00023_amd as kry
    import workloads as wk

    om = list(wl.omegas[args.omega_offset: args.omega_offset + args.n_omega])
    out, ys = precision_runs(wl, inp, dev, om, args.method, args.s_step_cli)
    if args.single_ref > 0:
        eps = torch.as_tensor(inp.eps, device=dev)
        sig = torch.as_tensor(inp.sigma, device=dev)
        b = torch.as_tensor(wk.source_vector(wl, om[0], 0.0)[None, :], device=dev)
        # the first frequencies solved again one at a time in FP64: a check
        # of the many-shift solves of both runs
        s = kry.Solver(eps, None, sig, kry.Options(storage="f64", krylov_dim=wl.krylov_dim, tol=1e-8,
                                                   s_step=args.s_step_cli))
        ref = []
        for k in range(min(args.single_ref, len(om))):
            y1 = s.solve_multifreq([om[k]], b, wl.T)[0]
            ref.append({name: float(torch.linalg.norm(ys[name][k] - y1) / torch.linalg.norm(y1))
                        for name in ("f32", "f64")})
            print(f"[bench] single omega {k} done", file=sys.stderr, flush=True)
        s.close()
        out["rel_err_vs_single_f64"] = ref
    print(json.dumps(out), flush=True)


def grad_transient_bench(args, wl, inp, dev):
    """Gradient of the flux of the field at time T (transient included) on
    the gradient workload's medium and frequencies, timed once after one
    untimed run, beside the time-averaged gradient of the same workload."""
    import torch

    import paper_1707_00023_amd as kry
    import workloads as wk

    eps = torch.as_tensor(inp.eps, device=dev)
    sig = torch.as_tensor(inp.sigma, device=dev)
    b = torch.as_tensor(wk.source_vector(wl, wl.omegas[0], 0.0)[None, :], device=dev)
    kf = wl.flux_plane
    s = kry.Solver(eps, None, sig, kry.Options(krylov_dim=wl.krylov_dim, tol=wl.tol, timing=True,
                                               s_step=args.s_step))
    out = {"metric": "finite-time flux gradient, time to solution", "workload": wl.name,
           "n": wl.n, "omegas": list(wl.omegas), "plane_k": kf, "T": args.grad_transient,
           "krylov_dim": wl.krylov_dim, "tol": wl.tol}
    for name, fn in (("time_averaged", lambda: s.grad(wl.omegas, b, kf)),
                     ("finite_time", lambda: s.grad_transient(wl.omegas, b, kf, args.grad_transient))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L, g = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = s.last_stats
        out[name] = {"s": dt, "loss": L, "grad_norm": float(torch.linalg.norm(g)),
                     "matvecs_stationary": st["matvecs_stationary"],
                     "matvecs_transient": st["matvecs_transient"],
                     "steps_transient": st["steps_transient"],
                     "ms_stationary": st["ms_stationary"], "ms_transient": st["ms_transient"]}
        print(f"[bench] gradient {name}: {dt:.2f} s", file=sys.stderr, flush=True)
    s.close()
    print(json.dumps(out), flush=True)


def other_methods(solver, wl, b, per_omega, split_stats, args):
    """The paper's other routes to the same y(T), each timed once on the same
    workload and solver after the split steps: the residual-restarted Krylov
    method (no shifted solve) and source splitting over subintervals of
    whole periods.  Reported with their relative difference from the split
    result of the last timed step (both are checked against the oracle in
    the tests)."""
    import torch
    y_split = solver.solve_multifreq(wl.omegas, b, wl.T, b_per_omega=per_omega)
    out = {}
    runs = [("restarted", lambda: solver.solve_restarted(wl.omegas, b, wl.T, b_per_omega=per_omega)),
            ("split2", lambda: solver.solve_split2(wl.omegas, b, wl.T, periods=args.split2_periods,
                                                   b_per_omega=per_omega))]
    for name, fn in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = solver.last_stats
        d = torch.linalg.norm(y - y_split, dim=1) / torch.linalg.norm(y_split, dim=1)
        out[name] = {"s": dt, "matvecs": st["matvecs_stationary"] + st["matvecs_transient"],
                     "restarts_or_steps": st["steps_transient"],
                     "err_estimate": st["max_err_estimate"],
                     "max_rel_diff_vs_split": float(d.max()),
                     "speedup_vs_split": (split_stats["ms_total"] / 1e3) / dt}
        print(f"[bench] {name}: {dt:.2f} s", file=sys.stderr, flush=True)
    if name == "split2":
        out["split2"]["periods_per_subinterval"] = args.split2_periods
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-batched", action="store_true",
                    help="batched workload only: time the block (batched) solve of a "
                         "column subset against plain one-column-at-a-time solves")
    ap.add_argument("--columns", type=int, default=8,
                    help="with --compare-batched: number of consecutive frequencies (one angle)")
    ap.add_argument("--omega-index", type=int, default=12,
                    help="with --compare-batched: first frequency index of the columns")
    ap.add_argument("--verbose", action="store_true",
                    help="library progress lines on stderr during long solves")
    ap.add_argument("--batched-modes", default="continuation",
                    help="with --compare-batched: modes compared with plain "
                         "(continuation, block)")
    ap.add_argument("--theta-index", type=int, default=0,
                    help="with --compare-batched: incidence angle index of the columns")
    ap.add_argument("--skip-plain", action="store_true",
                    help="with --compare-batched: time only the listed modes")
    ap.add_argument("--golden-check", action="store_true",
                    help="with --compare-batched on the batched workload: compare the solved "
                         "columns that have stored oracle values")
    ap.add_argument("--block-width", type=int, default=16)
    ap.add_argument("--block-steps", type=int, default=16)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--precision-compare", action="store_true",
                    help="FP32-storage solve of the first --n-omega frequencies against an "
                         "FP64 solve of the same columns on the GPU")
    ap.add_argument("--n-omega", type=int, default=2)
    ap.add_argument("--method", default="split", choices=["split", "restarted"],
                    help="precision compare: the split solver (Corollary 3) or the "
                         "residual-restarted method")
    ap.add_argument("--single-ref", type=int, default=0,
                    help="precision compare: also solve the first K frequencies one at a time "
                         "in FP64 and report both runs' errors against them")
    ap.add_argument("--omega-offset", type=int, default=0,
                    help="precision compare: index of the first frequency")
    ap.add_argument("--s-step", type=int, default=None,
                    help="s-step Arnoldi block size (default: the library binding's default)")
    ap.add_argument("--no-methods", action="store_true",
                    help="skip the one-off timings of the restarted method and source splitting")
    ap.add_argument("--no-multi-omega", action="store_true",
                    help="skip the one-off all-frequency runs of the 256^3 precision workload "
                         "(FP64 and FP32 storage, restarted method) after the 128^3 steps; "
                         "--no-methods skips them too")
    ap.add_argument("--split2-periods", type=int, default=5,
                    help="source splitting: periods of the source per subinterval")
    ap.add_argument("--stencil-planes", type=int, default=None, choices=[0, 4, 8, 16],
                    help="after the autotuner: force the basis stencil's form (0: cell-parallel, "
                         "4/8/16: z-marching with that many planes per workgroup)")
    ap.add_argument("--stencil-cells", type=int, default=None, choices=[1, 2, 4],
                    help="after the autotuner: force the cell-parallel basis stencil's cells per thread")
    ap.add_argument("--host-blocks", action="store_true",
                    help="finish each s-step block on the host (one synchronisation per "
                         "Gram-Schmidt pass) instead of on the device")
    ap.add_argument("--timing-sample", type=int, default=7, metavar="N",
                    help="time one kernel launch in N with HIP events inside the timed steps "
                         "(1: every launch, which adds about 4%% of host overhead to a solve)")
    ap.add_argument("--grad-transient", type=float, default=None, metavar="T",
                    help="time the gradient of the flux of the field at time T (transient "
                         "included) on the gradient workload (use with --workload c4)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="after the timed steps, one device copy of 1 GiB each way (the "
                         "reference dispatch that scales HBM counters to bytes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this solver has no multi-GPU path "
              "(the sharding design is documented, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1707_00023_amd as kry
    import workloads as wk

    wl = wk.CONFIGS[args.workload]
    inp = wk.generate(wl)
    dev = torch.device("cuda:0")
    args.s_step_cli = args.s_step
    if args.s_step is None:
        args.s_step = kry.DEFAULT_S_STEP
    if args.compare_batched:
        compare_batched(args, wl, inp, dev)
        return
    if args.precision_compare:
        precision_compare(args, wl, inp, dev)
        return
    if args.grad_transient is not None:
        grad_transient_bench(args, wl, inp, dev)
        return
    eps = torch.as_tensor(inp.eps, device=dev)
    sig = torch.as_tensor(inp.sigma, device=dev)
    solver = kry.Solver(eps, None, sig, kry.Options(storage=wl.storage, krylov_dim=wl.krylov_dim,
                                                    tol=wl.tol, timing=args.timing_sample,
                                                    s_step=args.s_step, host_blocks=args.host_blocks))
    tune = None if args.no_autotune else solver.autotune()
    if args.stencil_planes is not None or args.stencil_cells is not None:
        t = tune or {"cpt_stencil": 1, "cpt_update": 1, "cpt_dots": 1, "zm_stencil": 0}
        cells = args.stencil_cells if args.stencil_cells is not None else t["cpt_stencil"]
        planes = args.stencil_planes if args.stencil_planes is not None else t.get("zm_stencil", 0)
        solver.set_tune(cells, t["cpt_update"], t["cpt_dots"], planes)
        if tune is not None:
            tune = dict(tune, cpt_stencil=cells, zm_stencil=planes, forced=True)
    cols = [wk.source_vector(wl, w, float(th)) for w in wl.omegas for th in inp.thetas]
    b = torch.as_tensor(np.stack(cols), device=dev)
    per_omega = wl.n_theta > 1
    if not per_omega:
        b = b[: len(inp.thetas)]

    def step():
        return solver.solve_multifreq(wl.omegas, b, wl.T, b_per_omega=per_omega)

    for _ in range(args.warmup):
        step()
        print(f"[bench] warmup done {solver.last_stats['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(args.steps):
        step()
        stats.append(solver.last_stats)
        print(f"[bench] step {k} {solver.last_stats['ms_total']:.0f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1000.0 / args.steps
    calib = None
    if args.calibration_copy:
        # a device copy that moves exactly COPY_BYTES in and COPY_BYTES out:
        # the reference dispatch for scaling HBM counters to bytes
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1)
        calib = {"bytes_each_way": COPY_BYTES, "ms": cms, "gbs": 2 * COPY_BYTES / (cms * 1e6)}
        del src, dst

    # timed launches (one in --timing-sample per class, in launch order) and
    # every launch; a class's total time is estimated from its timed
    # launches' rate and all its bytes
    kms = np.sum([s["kernel_ms"] for s in stats], axis=0)
    kl = np.sum([s["kernel_launches"] for s in stats], axis=0)
    kb = np.sum([s["kernel_bytes"] for s in stats], axis=0)
    kla = np.sum([s["kernel_launches_all"] for s in stats], axis=0)
    kba = np.sum([s["kernel_bytes_all"] for s in stats], axis=0)
    kms_est = np.array([kms[i] * kba[i] / kb[i] if kb[i] > 0 else 0.0 for i in range(len(kms))])
    dom = int(np.argmax(kms_est))
    achieved = kb[dom] / (kms[dom] * 1e-3) / 1e9 if kms[dom] > 0 else 0.0
    last = stats[-1]
    matvecs = last["matvecs_stationary"] + last["matvecs_transient"]
    gcells = wl.N ** 3 * matvecs / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": "all-omega time-to-solution at 1e-8 rel err; HBM GB/s of curl SpMV+Arnoldi",
        "value": ms_per_step / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if wl.storage == "f64" else "f32-storage/f64-reductions",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{wl.N}^3", "unknowns": wl.n,
                   "n_omega": len(wl.omegas), "n_theta": wl.n_theta, "T": wl.T,
                   "krylov_dim": wl.krylov_dim, "tol": wl.tol, "s_step": args.s_step,
                   "parallelism": "single-gpu"},
        "gcell_updates_per_s": gcells,
        "matvecs": {"stationary": last["matvecs_stationary"], "transient": last["matvecs_transient"]},
        "phase_ms": {"stationary": last["ms_stationary"], "transient": last["ms_transient"]},
        "timing_sample": args.timing_sample,
        "kernels": {name: {"ms": float(kms_est[i]) / args.steps, "launches": int(kla[i]) // args.steps,
                           "timed_launches": int(kl[i]) // args.steps,
                           "bytes": float(kba[i]) / args.steps,
                           "gbs": float(kb[i] / (kms[i] * 1e-3) / 1e9) if kms[i] > 0 else 0.0}
                    for i, name in enumerate(kry.KERNEL_CLASSES)},
        "roofline": {"bound": "hbm", "kernel": kry.KERNEL_CLASSES[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "avg_launch_us": float(kms[dom] / max(kl[dom], 1) * 1e3),
                     "timed_launches": int(kl[dom]),
                     "alg_bytes_per_launch": float(kb[dom] / max(kl[dom], 1)),
                     "traffic": measured_traffic(kry.KERNEL_CLASSES[dom], args.workload,
                                                 float(kb[dom] / max(kl[dom], 1)))},
        "launch_shapes": tune,
        "converged": bool(last["converged"]),
        "max_residual": last["max_residual"],
        "max_err_estimate": last["max_err_estimate"],
    }
    # curl + Arnoldi together: operator, Gram, update and combination kernels
    agg = [i for i, k in enumerate(kry.KERNEL_CLASSES) if kms[i] > 0]
    agg_ms = float(sum(kms[i] for i in agg))
    agg_b = float(sum(kb[i] for i in agg))
    out["curl_arnoldi"] = {"gbs": agg_b / (agg_ms * 1e-3) / 1e9 if agg_ms > 0 else 0.0,
                           "frac": agg_b / (agg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if agg_ms > 0 else 0.0,
                           "ms_per_step": float(sum(kms_est[i] for i in agg)) / args.steps,
                           "kernels": [kry.KERNEL_CLASSES[i] for i in agg]}
    if not args.no_methods:
        out["methods"] = other_methods(solver, wl, b, per_omega, stats[-1], args)
    if not args.no_methods and not args.no_multi_omega and args.workload == "c2":
        # every frequency of the 256^3 precision workload (16 on one shared
        # source), timed once in each storage type by the restarted method
        solver.close()
        wl5 = wk.CONFIGS["c5"]
        om5 = list(wl5.omegas)
        print(f"[bench] all {len(om5)} frequencies of {wl5.name}", file=sys.stderr, flush=True)
        r5, _ = precision_runs(wl5, wk.generate(wl5), dev, om5, "restarted", args.s_step_cli, verbose=False)
        out["all_omega_multi"] = {
            "workload": wl5.name, "grid": f"{wl5.N}^3", "unknowns": wl5.n, "n_omega": len(om5),
            "T": wl5.T, "krylov_dim": wl5.krylov_dim, "method": "restarted",
            "f64": {k: r5["f64"][k] for k in ("tol", "s", "matvecs_transient", "converged")},
            "f32": {k: r5["f32"][k] for k in ("tol", "s", "matvecs_transient", "converged")},
            "max_rel_err_f32_vs_f64": max(r5["rel_err_per_omega"]),
            "speedup_f32_over_f64": r5["speedup_f32_over_f64"]}
    if calib is not None:
        out["calibration_copy"] = calib
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, inp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
