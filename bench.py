"""Benchmark: APG solves/s and p50/p99 solve latency at a fixed dual tolerance.

One step is one full solve of a scenario-tree stochastic MPC instance to the
tolerance: the per-solve data step, every APG iteration (backward sweep,
forward sweep with the fused prox/dual update and residual, Nesterov
extrapolation, stop test) and the final cost evaluation, starting from a
zero dual.  The offline factor step and the step size (power iteration for
the Lipschitz constant, cached per tree) run before the timed region and are
reported separately.

Default workload ``dwn128``: a synthetic network with the paper's dimensions
(63 tanks, 114 pumps/valves, 88 demands, 17 mixing nodes), horizon 24, a
tree branching 4 then 2 up to 128 scenarios (K = 2429 nodes), FP64, run to a
residual of 1e-4.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "APG solves/sec and p50/p99 solve latency at fixed dual tolerance, 1 MI355X"
HBM_PEAK_GBS = 8000.0


def sweep_bytes(nx, nu, elem, K, n_blocks, kind, form):
    """Algorithmic HBM bytes of one sweep direction over one iteration.

    Backward, per node: y and y_prev (2 (2nx+nu)), kappa (nu) read, j (P in
    the scan form, nu) written.  Forward, per node: j (nu), 1/p, g (nx), y and
    y_prev read, u (nu), x (nx) and y_next (2nx+nu) written; the scan form
    also reads kappa - Pi kappa (nu).  Children and parents inside a
    workgroup's subtree stay on chip (the scan form's forward launch re-reads
    the ancestors of a workgroup's nodes: not counted).  With the stage
    factors in registers each distinct block (nu^2) is read once; the
    projector and scan forms read only the small CSRs of G and E'."""
    if kind == "bwd":
        per_node = 4 * nx + 4 * nu
    else:
        per_node = 8 * nx + (6 if form == "scan" else 5) * nu + 1
    factors = n_blocks * nu * nu if form == "segment" else 0
    return (per_node * K + factors) * elem


KERNEL_SOURCES = ("paper_1904_10548_amd/csrc/segment_kernels.hip",
                  "paper_1904_10548_amd/csrc/scan_kernels.hip",
                  "paper_1904_10548_amd/csrc/seg_device.h",
                  "paper_1904_10548_amd/csrc/kernels.h")


def kernel_prefix(form):
    return "scan" if form == "scan" else "seg"


# The schedule settings that shape each sweep's launches: the backward
# launches do not depend on the forward launch's grouping, nor the forward
# launch on light upper levels.
SPEC_KEYS = {"bwd": ("TAPG_SCAN", "TAPG_LEVELS", "TAPG_TOP"),
             "fwd": ("TAPG_SCAN", "TAPG_LEVELS", "TAPG_FWD_GROUP")}


def _spec_items(spec, kind):
    d = dict(kv.split("=", 1) for kv in spec.split())
    return {k: d.get(k) for k in SPEC_KEYS[kind]}


def measured_traffic(workload, precision, form, spec=None, kind=None):
    """HBM bytes per launch of each sweep kind (or of ``kind`` alone) from the
    committed FETCH_SIZE / WRITE_SIZE counter summary, if it was taken on this
    workload, sweep form and schedule (the settings ``spec``; with ``kind``
    only those that shape that sweep's launches) with the current kernel
    sources (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles",
                        f"{kernel_prefix(form)}_sweeps_{workload}_{precision}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    line = next((l for l in open(path) if l.startswith("traffic-json:")), None)
    if line is None:
        return None
    data = json.loads(line.split(":", 1)[1])
    sha = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            sha.update(fh.read())
    if data.get("kernel_sources_sha256") != sha.hexdigest():
        return None
    taken = data.get("spec", "")
    if kind is not None:
        if spec is not None and _spec_items(taken, kind) != _spec_items(spec, kind):
            return None  # taken under another schedule: other launches
        return data["bytes_per_launch"].get(kind)
    if spec is not None and sorted(taken.split()) != sorted(spec.split()):
        return None
    return data["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="dwn128")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iter", type=int, default=400000)
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the planner's schedule and the default sweep form (profiling runs)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: offered requests/s")
    ap.add_argument("--rates", default="", help="serve: comma-separated offered rates (load curve)")
    ap.add_argument("--requests", type=int, default=2000,
                    help="serve: timed requests (per offered rate)")
    ap.add_argument("--sessions", type=int, default=32, help="serve: sessions (one tree each)")
    ap.add_argument("--max-batch", type=int, default=64, help="serve: trees in flight")
    ap.add_argument("--hbm-gb", type=float, default=64.0, help="serve: admission budget")
    ap.add_argument("--horizon-steps", type=int, default=168, help="closed loop: H_s")
    ap.add_argument("--ext-steps", type=int, default=2,
                    help="timed steps of each extension workload in the default run")
    ap.add_argument("--dense-wu", action="store_true",
                    help="single tree with a dense W_u (100 I + a seeded rank-8 coupling)")
    ap.add_argument("--no-extensions", action="store_true",
                    help="time the headline workload only")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1 "
                          "(sharding a tree or a batch across GPUs is not built)"}))
        sys.exit(2)

    import dwn_synth as ds
    from paper_1904_10548_amd import tapg

    try:
        import torch
        have_torch = torch.cuda.is_available()
    except Exception:  # torch is optional plumbing here
        have_torch = False

    # long solves print their own progress (iterations, trees running) to stderr
    os.environ.setdefault("TAPG_PROGRESS", "30")
    if args.config == "batch64":
        out = main_batch(args, ds, tapg)
        print(json.dumps(out), flush=True)
        return
    if args.config == "serve":
        return main_serve(args, ds, tapg)
    if args.config == "closed_loop":
        print(json.dumps(main_closed_loop(args, ds, tapg)), flush=True)
        return
    out = main_single(args, ds, tapg, have_torch)
    if not args.no_extensions and args.config == "dwn128":
        out["extensions"] = extensions(args, ds, tapg, have_torch)
    print(json.dumps(out), flush=True)


def extensions(args, ds, tapg, have_torch):
    """The extension workloads, timed in the same run as the headline (each a
    few steps at the paper's tolerance 5e-2): the 2,048-scenario tree and the
    64-tree batch in FP64 and FP32 sweeps, the 128-scenario tree with a dense
    W_u, and a closed loop."""
    ext = {}
    for cfg, prec in (("dwn2048", "fp64"), ("dwn2048", "fp32"), ("batch64", "fp64"),
                      ("batch64", "fp32")):
        a = argparse.Namespace(**vars(args))
        a.config, a.precision, a.tol = cfg, prec, 5e-2
        a.steps, a.warmup = args.ext_steps, 1
        a.no_cpu_baseline = True
        a.max_iter = 400000
        print(f"[bench] extension {cfg} {prec} tol 5e-2", file=sys.stderr, flush=True)
        r = main_batch(a, ds, tapg) if cfg == "batch64" else main_single(a, ds, tapg, have_torch)
        ext[f"{cfg}_{prec}_tol5e-2"] = {k: r[k] for k in r if k not in (
            "metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data",
            "cpu_baseline")}
    # the general path: a dense W_u (dense stage factors in registers)
    a = argparse.Namespace(**vars(args))
    a.config, a.precision, a.tol, a.dense_wu = "dwn128", "fp64", 5e-2, True
    a.steps, a.warmup, a.no_cpu_baseline, a.max_iter = args.ext_steps, 1, True, 400000
    print("[bench] extension dwn128 dense W_u fp64 tol 5e-2", file=sys.stderr, flush=True)
    r = main_single(a, ds, tapg, have_torch)
    ext["dwn128_dense_wu_fp64_tol5e-2"] = {k: r[k] for k in r if k not in (
        "metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "cpu_baseline")}
    a = argparse.Namespace(**vars(args))
    a.config, a.precision, a.tol, a.dense_wu = "dwn128", "fp64", 5e-2, False
    print("[bench] extension closed loop", file=sys.stderr, flush=True)
    r = main_closed_loop(a, ds, tapg)
    ext["closed_loop_dwn128_fp64_tol5e-2"] = {k: r[k] for k in r if k not in (
        "metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "cpu_baseline")}
    return ext


def main_single(args, ds, tapg, have_torch):
    """One tree (dwn128, dwn2048 or small) solved to the tolerance per step."""
    if have_torch:
        import torch
    P = ds.config_problem(args.config)
    if args.dense_wu:  # the general path: dense stage factors, no projector or scan form
        P.weights.W_u = ds.dense_input_weight(P.net.nu)
    net, w = P.net, P.weights
    prec = tapg.TAPG_FP64 if args.precision == "fp64" else tapg.TAPG_FP32
    elem = 8 if prec == tapg.TAPG_FP64 else 4
    t0 = time.perf_counter()
    S = tapg.Solver(dict(A=net.A, B=net.B, Gd=net.Gd, E=net.E, Ed=net.Ed, xmin=net.xmin,
                         xmax=net.xmax, xs=net.xs, umin=net.umin, umax=net.umax),
                    dict(W_alpha=w.W_alpha, W_s=w.W_s, W_x=w.W_x, alpha0=w.alpha0,
                         c_energy=w.c_energy, W_u=w.W_u),
                    P.tree.N, gamma=0.0, tol=args.tol, max_iter=args.max_iter,
                    check_every=args.check_every, precision=prec)
    factor_s = time.perf_counter() - t0
    _, n_blocks = tapg.tapg_factor_blocks(S.h, P.tree.N)
    tree = S.add_tree(P.tree.nodes_per_stage, P.tree.anc, P.tree.prob, P.data.demand,
                      P.data.price)
    t0 = time.perf_counter()
    L = tapg.tapg_estimate_lipschitz(S.h, tree, 100)
    lipschitz_s = time.perf_counter() - t0
    # schedule and sweep form picked by the autotuner (setup, not timed)
    t0 = time.perf_counter()
    tune_ms, tune_nc = (None, 0) if args.no_autotune else tapg.tapg_autotune(S.h, [tree], 100)
    tune_s = time.perf_counter() - t0
    if args.no_autotune:
        S.solve(tree, P.p, P.q)  # the slot exists once solved
    form, n_bwd = tapg.tapg_sweep_form(S.h, [tree])
    spec = tapg.tapg_schedule_spec(S.h, [tree])
    print(f"[bench] schedule {spec}", file=sys.stderr, flush=True)
    print(f"[bench] {args.config} K={P.tree.K} L={L:.6g} factor {factor_s:.3f}s "
          f"power {lipschitz_s:.3f}s autotune {tune_s:.3f}s: {form} form, {n_bwd} backward "
          f"launches, {tune_ms} ms/iter", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        st, u0, res = S.solve(tree, P.p, P.q)
        print(f"[bench] warmup {i}: iters={res.iters} res={res.primal_res:.3e} "
              f"{res.solve_ms:.1f} ms", file=sys.stderr, flush=True)

    if have_torch:
        torch.cuda.synchronize()
    lat = []
    results = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        st, u0, res = S.solve(tree, P.p, P.q)
        lat.append(time.perf_counter() - t1)
        results.append(res.as_dict())
        print(f"[bench] step {i}: iters={res.iters} res={res.primal_res:.3e} "
              f"cost={res.cost:.10g} {lat[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    if have_torch:
        torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    lat_ms = np.array(lat) * 1e3
    iters = results[-1]["iters"]

    roof = None
    kt = None
    if not args.no_kernel_timing:
        # Device time of every sweep-kernel launch, HIP events on the solver's
        # stream, over one more solve of the same workload; each launch's event
        # pair also reads the dispatch cost of an empty launch (measured the
        # same way), which is taken off.
        tapg.tapg_kernel_timing(S.h, True)
        S.solve(tree, P.p, P.q)
        kt = tapg.tapg_kernel_times(S.h)
        tapg.tapg_kernel_timing(S.h, False)
        pair_us = tapg.tapg_event_pair_overhead(S.h)
        kinds = {}
        for kind in ("bwd", "fwd"):
            ms_raw, n = kt[kind]
            ms = ms_raw - n * pair_us * 1e-3
            b_iter = sweep_bytes(net.nx, net.nu, elem, P.tree.K, n_blocks, kind, form)
            its = iters  # one timed solve of the same workload
            kinds[kind] = dict(ms=ms, launches=n, bytes=b_iter * its, avg_us=1e3 * ms / max(n, 1),
                               avg_us_raw=1e3 * ms_raw / max(n, 1))
        dom = max(kinds, key=lambda k: kinds[k]["ms"])
        d = kinds[dom]
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        # measured HBM bytes per launch of the dominant kernel (FETCH_SIZE +
        # WRITE_SIZE, calibrated against a plain copy) from the committed
        # counter summary, when it matches these kernel sources
        tb = measured_traffic(args.config, args.precision, form, spec, kind=dom)
        traffic = round(tb) if tb is not None else None
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "traffic_unit": "HBM bytes per launch",
                "traffic_gbs": None if traffic is None else
                round(traffic / (d["avg_us"] * 1e-6) / 1e9, 2),
                "traffic_over_algorithmic": None if traffic is None else
                round(traffic / (d["bytes"] / max(d["launches"], 1)), 3),
                "kernel": f"{kernel_prefix(form)}_{dom}_kernel", "avg_launch_us": round(d["avg_us"], 3),
                "avg_launch_us_event_pairs": round(d["avg_us_raw"], 3),
                "event_pair_overhead_us": round(pair_us, 3),
                "bytes_per_launch": round(d["bytes"] / max(d["launches"], 1), 1),
                "other": {k: {"avg_launch_us": round(v["avg_us"], 3),
                              "avg_launch_us_event_pairs": round(v["avg_us_raw"], 3),
                              "launches": v["launches"],
                              "ms": round(v["ms"], 3)} for k, v in kinds.items()},
                "iteration_end_ms": round(kt["end"][0], 3)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(P, results[-1]["gamma"], iters, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(args.steps / total, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == tapg.TAPG_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: nx={net.nx} nu={net.nu} nd={net.nd} "
                               f"ns={net.ns} N={P.tree.N}, "
                               f"{P.tree.n_scenarios} scenarios, K={P.tree.K}, "
                               f"W_u={wu_text(w.W_u)}, tol={args.tol:g}, cold start",
                   "K": P.tree.K, "N": P.tree.N, "tol": args.tol, "precision": args.precision},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "iters": iters,
        "ms_per_iter": round(float(np.median(lat_ms)) / max(iters, 1), 5),
        "final_residual": results[-1]["primal_res"],
        "cost": results[-1]["cost"],
        "factor_step_s": round(factor_s, 4),
        "factor_blocks": n_blocks,
        "lipschitz_s": round(lipschitz_s, 4),
        "schedule": {"form": form, "bwd_launches": n_bwd, "spec": spec,
                     "autotune_s": round(tune_s, 3), "autotune_candidates": tune_nc,
                     "autotune_ms_per_iter": None if tune_ms is None else round(tune_ms, 5)},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    S.close()
    return out


def wu_text(W):
    d = float(W[0, 0])
    return f"{d:g} I" if np.array_equal(W, d * np.eye(W.shape[0])) else "dense"


def main_batch(args, ds, tapg):
    """64 trees of 16..256 scenarios (K from 349 to 4,605) on the Barcelona-sized
    network, all solved by one tapg_batch_solve per step (cold start, each tree
    to the tolerance with its own step size).  Value: trees solved per second."""
    trees_p = [ds.config_problem("batch64", i) for i in range(64)]
    P0 = trees_p[0]
    net, w = P0.net, P0.weights
    prec = tapg.TAPG_FP64 if args.precision == "fp64" else tapg.TAPG_FP32
    S = tapg.Solver(dict(A=net.A, B=net.B, Gd=net.Gd, E=net.E, Ed=net.Ed, xmin=net.xmin,
                         xmax=net.xmax, xs=net.xs, umin=net.umin, umax=net.umax),
                    dict(W_alpha=w.W_alpha, W_s=w.W_s, W_x=w.W_x, alpha0=w.alpha0,
                         c_energy=w.c_energy, W_u=w.W_u),
                    P0.tree.N, gamma=0.0, tol=args.tol, max_iter=args.max_iter,
                    check_every=args.check_every, precision=prec)
    trees = [S.add_tree(P.tree.nodes_per_stage, P.tree.anc, P.tree.prob, P.data.demand,
                        P.data.price) for P in trees_p]
    ps, qs = [P.p for P in trees_p], [P.q for P in trees_p]
    K_tot = sum(P.tree.K for P in trees_p)
    t0 = time.perf_counter()
    for t in trees:
        tapg.tapg_estimate_lipschitz(S.h, t, 100)
    lipschitz_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    if args.no_autotune:  # the planner's schedule (or the one TAPG_* settings force)
        tune_ms, tune_nc = None, 0
        S.batch_solve(trees, ps, qs)  # the schedule is built with the first solve
    else:
        tune_ms, tune_nc = tapg.tapg_autotune(S.h, trees, 10)
    tune_s = time.perf_counter() - t0
    form, n_bwd = tapg.tapg_sweep_form(S.h, trees)
    spec = tapg.tapg_schedule_spec(S.h, trees)
    elem = 8 if prec == tapg.TAPG_FP64 else 4
    forest_bytes = sum(sweep_bytes(net.nx, net.nu, elem, K_tot, 1, kind, form) for kind in ("bwd", "fwd"))
    print(f"[bench] batch64: 64 trees, {K_tot} nodes, power {lipschitz_s:.3f}s, autotune "
          f"{tune_s:.3f}s: {form} form, {n_bwd} backward launches, {tune_ms} ms/iter",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        st, _, res = S.batch_solve(trees, ps, qs)
        print(f"[bench] warmup {i}: iters {min(r.iters for r in res)}..{max(r.iters for r in res)} "
              f"{res[0].solve_ms:.1f} ms", file=sys.stderr, flush=True)
    lat, last = [], None
    t_start = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        st, _, res = S.batch_solve(trees, ps, qs)
        lat.append(time.perf_counter() - t1)
        last = res
        print(f"[bench] step {i}: iters {min(r.iters for r in res)}..{max(r.iters for r in res)} "
              f"{lat[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_start
    lat_ms = np.array(lat) * 1e3
    iters = [r.iters for r in last]
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the largest tree, scaled to the batch's total iterations x nodes
        big = max(range(64), key=lambda k: trees_p[k].tree.K)
        cb = cpu_baseline(trees_p[big], last[big].gamma, iters[big], args.cpu_seconds)
        work_big = iters[big] * trees_p[big].tree.K
        work_all = sum(it * P.tree.K for it, P in zip(iters, trees_p))
        per_solve_s = (1.0 / cb["value"]) * work_all / work_big
        cpu = {"value": round(64.0 / per_solve_s, 6), "unit": "trees/s", "cores": cb["cores"],
               "kind": "oracle",
               "sample": cb["sample"] + f"; scaled by node-iterations to all 64 trees "
                                        f"({work_all} node-iterations)"}
    out = {
        "metric": METRIC + " (64-tree batch)",
        "value": round(64 * args.steps / total, 4),
        "unit": "trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == tapg.TAPG_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"batch64: 64 trees, S in 16..256, K total {K_tot}, "
                               f"W_u={wu_text(w.W_u)}, tol={args.tol:g}, cold start, "
                               f"one tapg_batch_solve per step",
                   "trees": 64, "K_total": K_tot, "tol": args.tol, "precision": args.precision},
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "iters_min": int(min(iters)), "iters_max": int(max(iters)),
        "converged": int(sum(r.converged for r in last)),
        "lipschitz_s": round(lipschitz_s, 4),
        # one iteration of the whole forest (every tree running), as the
        # autotuner timed it with the schedule and form it kept
        "schedule": {"form": form, "bwd_launches": n_bwd, "spec": spec,
                     "autotune_s": round(tune_s, 3), "autotune_candidates": tune_nc,
                     "forest_gb_per_iter": round(forest_bytes / 1e9, 4)},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    if tune_ms is not None:
        # the forest's whole iteration (every launch) as the autotuner timed it
        # with all trees running, against the HBM peak
        gbs = forest_bytes / (tune_ms * 1e-3) / 1e9
        out["schedule"].update(forest_ms_per_iter=round(tune_ms, 5), forest_gbs=round(gbs, 1))
        out["roofline"] = {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": None,
                           "kernel": "forest iteration (every launch)",
                           "bytes_per_iteration": int(forest_bytes),
                           "ms_per_iteration": round(tune_ms, 5)}
    S.close()
    return out


def main_closed_loop(args, ds, tapg):
    """Closed-loop receding-horizon simulation (Sec. 6.3): H_s = 168 hourly
    steps on the 128-scenario tree, each solved to the tolerance warm started
    from the previous dual; the paper's indices KPI_E, KPI_S and KPI_tau (the
    worst solve time)."""
    P = ds.config_problem("dwn128")
    net, w = P.net, P.weights
    prec = tapg.TAPG_FP64 if args.precision == "fp64" else tapg.TAPG_FP32
    H = args.horizon_steps
    inp = ds.make_loop_inputs(net, H + P.tree.N, seed=1006)
    S = tapg.Solver(dict(A=net.A, B=net.B, Gd=net.Gd, E=net.E, Ed=net.Ed, xmin=net.xmin,
                         xmax=net.xmax, xs=net.xs, umin=net.umin, umax=net.umax),
                    dict(W_alpha=w.W_alpha, W_s=w.W_s, W_x=w.W_x, alpha0=w.alpha0,
                         c_energy=w.c_energy, W_u=w.W_u),
                    P.tree.N, gamma=0.0, tol=args.tol, max_iter=args.max_iter,
                    check_every=args.check_every, precision=prec)
    tree = S.add_tree(P.tree.nodes_per_stage, P.tree.anc, P.tree.prob, P.data.demand,
                      P.data.price)
    tapg.tapg_estimate_lipschitz(S.h, tree, 100)
    tapg.tapg_autotune(S.h, [tree], 100)
    def forecast(k):
        if k % 24 == 0:
            print(f"[bench] closed loop: step {k} of {H}", file=sys.stderr, flush=True)
        return inp.tree_data(net, P.tree, k)

    t0 = time.perf_counter()
    xt, ut, tau, its, st = tapg.tapg_closed_loop(S.h, tree, H, P.p, P.q, forecast, P.tree.K,
                                                 net.nd)
    total = time.perf_counter() - t0
    out = {
        "metric": METRIC + " (closed loop)",
        "value": round(H / total, 4),
        "unit": "steps/s",
        "n_gpus": 1, "steps": H, "warmup": 0,
        "ms_per_step": round(1e3 * total / H, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == tapg.TAPG_FP64 else "f32", "data": "synthetic",
        "config": {"workload": f"closed loop: dwn128 tree (K={P.tree.K}), H_s={H} hourly steps, "
                               f"W_u={wu_text(w.W_u)}, tol={args.tol:g}, warm-started re-solves",
                   "H_s": H, "tol": args.tol, "precision": args.precision},
        "kpi_E": round(st.kpi_E, 6), "kpi_S": round(st.kpi_S, 6),
        "kpi_tau_ms": round(st.kpi_tau_ms, 3), "mean_tau_ms": round(st.mean_tau_ms, 3),
        "p50_ms": round(float(np.percentile(tau, 50)), 3),
        "p99_ms": round(float(np.percentile(tau, 99)), 3),
        "iters_first": int(its[0]), "iters_p50": int(np.percentile(its, 50)),
        "iters_max": int(its.max()), "steps_converged": int(st.steps_converged),
        "max_viol_box": st.max_viol_box, "max_viol_eq": st.max_viol_eq,
        "roofline": None, "cpu_baseline": None,
    }
    S.close()
    return out


def main_serve(args, ds, tapg):
    """Serving loop: Poisson arrivals of receding-horizon re-solves over
    `sessions` trees of 32..512 scenarios (K 669..8,701); each request starts
    from its session's previous root input (q) and a drifted state (p), is warm
    started when its session's previous request solved the same tree, and is
    admitted into the running set by HBM budget (continuous batching).
    Value: requests completed per second over the timed requests; latency is
    submit to completion.  With --rates r1,r2,... the same server is driven at
    each offered rate in turn (a load curve); the line's value is the last
    rate's."""
    import threading
    n_sess = args.sessions
    sess = [ds.config_problem("serve", i) for i in range(n_sess)]
    P0 = sess[0]
    net, w = P0.net, P0.weights
    prec = tapg.TAPG_FP64 if args.precision == "fp64" else tapg.TAPG_FP32
    S = tapg.Solver(dict(A=net.A, B=net.B, Gd=net.Gd, E=net.E, Ed=net.Ed, xmin=net.xmin,
                         xmax=net.xmax, xs=net.xs, umin=net.umin, umax=net.umax),
                    dict(W_alpha=w.W_alpha, W_s=w.W_s, W_x=w.W_x, alpha0=w.alpha0,
                         c_energy=w.c_energy, W_u=w.W_u),
                    P0.tree.N, gamma=0.0, tol=args.tol, max_iter=args.max_iter,
                    check_every=args.check_every, precision=prec)
    trees = [S.add_tree(P.tree.nodes_per_stage, P.tree.anc, P.tree.prob, P.data.demand,
                        P.data.price) for P in sess]
    K_of = [int(P.tree.K) for P in sess]
    t0 = time.perf_counter()
    for t in trees:
        tapg.tapg_estimate_lipschitz(S.h, t, 100)
    print(f"[bench] serve: {n_sess} sessions, K {min(K_of)}..{max(K_of)}, "
          f"power {time.perf_counter() - t0:.2f}s", file=sys.stderr, flush=True)
    srv = tapg.tapg_server_create(S.h, int(args.hbm_gb * 2**30), args.max_batch)
    rng = np.random.default_rng(np.random.SeedSequence([1004, 17]))
    last_q = [P.q.copy() for P in sess]
    last_p = [P.p.copy() for P in sess]
    lock = threading.Lock()

    def run(reqs, rate):
        """Submit `reqs` requests (Poisson at `rate`, or all at once if rate is
        None) round-robin over the sessions; returns per-request results."""
        gaps = rng.exponential(1.0 / rate, size=reqs) if rate else np.zeros(reqs)
        drift = rng.normal(0.0, 0.05, size=(reqs, net.nx))
        tickets, results = [None] * reqs, [None] * reqs
        submit_t, done_t = [0.0] * reqs, [0.0] * reqs

        def collector():
            for i in range(reqs):
                while tickets[i] is None:
                    time.sleep(0.0005)
                st, u0, r, lat = tapg.tapg_server_poll(srv, tickets[i], net.nu, -1)
                done_t[i] = time.perf_counter()
                k = i % n_sess
                with lock:
                    if st in (tapg.TAPG_OK, tapg.TAPG_ENOTCONV):
                        last_q[k] = np.clip(u0, net.umin, net.umax)
                results[i] = (st, r, lat)

        th = threading.Thread(target=collector)
        th.start()
        t_next = time.perf_counter()
        for i in range(reqs):
            t_next += gaps[i]
            while time.perf_counter() < t_next:
                time.sleep(max(0.0, min(0.001, t_next - time.perf_counter())))
            k = i % n_sess
            with lock:
                if rate:
                    last_p[k] = np.clip(last_p[k] + drift[i], net.xmin + 0.5, net.xmax - 0.5)
                p, q = last_p[k].copy(), last_q[k].copy()
            submit_t[i] = time.perf_counter()
            tickets[i] = tapg.tapg_server_submit(srv, trees[k], p, q, session=k)
        th.join()
        return results, submit_t, done_t

    # the first (cold) request of every session completes before the timed
    # arrivals start, so the timed windows see the warm-started re-solves only
    run(n_sess, None)
    # and one untimed round of re-solves at once: the first re-solve after a
    # cold solve moves q the most and needs the most iterations
    run(n_sess, 1e6)
    print(f"[bench] serve: {n_sess} cold requests and one re-solve each done", file=sys.stderr,
          flush=True)
    rates = [float(r) for r in args.rates.split(",")] if args.rates else [args.rate]
    curve = []
    for rate in rates:
        stats0, timing0 = tapg.tapg_server_stats(srv), tapg.tapg_server_timing(srv)
        results, submit_t, done_t = run(args.requests, rate)
        stats, timing = tapg.tapg_server_stats(srv), tapg.tapg_server_timing(srv)
        stats = {k: stats[k] - stats0[k] for k in ("batches", "solved", "busy_ms")}
        timing = {k: timing[k] - timing0[k] for k in timing}
        lat_ms = np.array([r[2] for r in results])
        iters = np.array([r[1].iters for r in results])
        node_iters = float(sum(r[1].iters * K_of[i % n_sess] for i, r in enumerate(results)))
        window = max(done_t) - min(submit_t)
        done_rate = args.requests / window
        point = {
            "offered_rate": rate, "completed_rate": round(done_rate, 2),
            "p50_ms": round(float(np.percentile(lat_ms, 50)), 2),
            "p99_ms": round(float(np.percentile(lat_ms, 99)), 2),
            "mean_ms": round(float(lat_ms.mean()), 2),
            # Little's law: requests in the system on average
            "mean_in_system": round(done_rate * float(lat_ms.mean()) / 1e3, 2),
            "completed_ok": int(sum(r[0] in (tapg.TAPG_OK, tapg.TAPG_ENOTCONV) for r in results)),
            "converged": int(sum(bool(r[1].converged) for r in results)),
            "iters_p50": int(np.percentile(iters, 50)), "iters_mean": round(float(iters.mean()), 1),
            "iters_max": int(iters.max()),
            # device work: node-iterations of the requests, and their rate while
            # the worker ran chunks (the forest's throughput on this mix)
            "node_iters_per_request": round(node_iters / args.requests),
            "node_iters_per_chunk_s": round(node_iters / (stats["busy_ms"] / 1e3))
            if stats["busy_ms"] > 0 else None,
            "forests_formed": stats["batches"],
            "worker_ms": {k: round(v, 1) for k, v in timing.items()},
            "worker_busy_frac": round(sum(timing.values()) / (1e3 * window), 3),
        }
        curve.append(point)
        print(f"[bench] serve: {json.dumps(point)}", file=sys.stderr, flush=True)
    tapg.tapg_server_destroy(srv)
    last = curve[-1]
    out = {
        "metric": METRIC + " (serving)",
        "value": last["completed_rate"],
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": args.requests,
        "warmup": n_sess,
        "ms_per_step": round(1e3 / last["completed_rate"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == tapg.TAPG_FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"serve: Poisson {rates[-1]:g} req/s offered, {n_sess} sessions, "
                               f"S in 32..512, tol={args.tol:g}, warm-started re-solves, "
                               f"continuous batching (max {args.max_batch} in flight, "
                               f"{args.hbm_gb:g} GB admission budget)",
                   "offered_rate": rates[-1], "requests": args.requests, "sessions": n_sess,
                   "tol": args.tol, "precision": args.precision},
        "p50_ms": last["p50_ms"], "p99_ms": last["p99_ms"],
        "curve": curve,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    S.close()


def cpu_baseline(P, gamma, gpu_iters, seconds):
    """The FP64 oracle on the host: time a bounded number of its iterations and
    scale to the iteration count of one solve."""
    import oracle as O

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")),
                         "unknown")
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    f = O.StageFactors(P.net, P.weights.W_u, P.tree)
    t0 = time.perf_counter()
    O.apg(P, gamma, f, 3)
    per = (time.perf_counter() - t0) / 3
    n = max(3, min(gpu_iters, int(seconds / max(per, 1e-6))))
    t0 = time.perf_counter()
    O.apg(P, gamma, f, n)
    per = (time.perf_counter() - t0) / n
    return {"value": round(1.0 / (per * gpu_iters), 6), "unit": "solves/s", "cores": threads,
            "kind": "oracle", "cpu_model": model, "nproc": os.cpu_count(),
            "usable_cpus": usable,
            "sample": f"{n} oracle APG iterations (NumPy FP64, per-stage einsum) on the same "
                      f"instance; per-iteration time {per * 1e3:.2f} ms scaled to the "
                      f"{gpu_iters} iterations of one solve"}


if __name__ == "__main__":
    main()
