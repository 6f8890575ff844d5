#!/usr/bin/env python3
"""Benchmark: DOF-RHS evaluations per second of the DGSEM Euler step on one MI355X.

Workload (default): 3D compressible Euler, Taylor-Green vortex at Mach 0.1 with a seeded 1 %
smooth density perturbation, DGSEM N = 3 on 32^3 periodic hex elements ([-pi, pi]^3), EC
flux-differencing volume integral + LLF surface flux, Carpenter-Kennedy 5-stage RK with the
CFL 0.5 time step, float64.  A timed step is one full RK step (time step + 5 stages of
interface fluxes and volume/lift/Jacobian/stage update), inputs resident in HBM.

value = steps * 5 * E * (N+1)^3 / seconds (the paper's PID, Eq. (3), is 1/value).
Timing: a warm-up of at least 0.5 s of steps, then 5 repetitions of exactly --steps steps on
the product path (dgx_step replaying its captured step-pair graph); `value` is from the
fastest repetition (the paper's best-of-5 rule, Section 3.1), `value_median` from the median.
The stage kernel's average launch duration for the roofline comes from a separate pass with
HIP events on the handle's stream.
Also reported: the right-hand side alone, the mixed-precision and the ensemble variants,
the roofline of the dominant kernel and the oracle on the host.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-RHS evals/sec (PID) 3D Euler N=3, FP64 vs mixed vs batched, 1 MI355X"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CUs x 2.4 GHz x 128 FP64 flops per clock
# vector-instruction issue: 1024 SIMDs x 2.4 GHz, one 64-lane instruction per 4 clocks
# (16 lanes a clock; float64 FMAs and 32-bit operations alike)
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4
FP64_PEAK_TFLOPS = 78.6


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_state(solver, name):
    import torch

    from paper_2108_06476_amd import inputs
    if name.startswith("tgv"):
        return inputs.tgv(solver.node_coords()).contiguous()   # evaluated on the GPU
    xyz = solver.node_coords().cpu().numpy()
    if name.startswith("sedov"):
        u = inputs.sedov(xyz)
    else:
        u = inputs.density_wave(xyz)
    return torch.from_numpy(u).cuda()


WARMUP_FLOOR_S = 0.5   # warm-up runs at least this long, whatever --warmup says
REPS = 5               # timed repetitions: the paper's best of 5 (Section 3.1), plus the median


def warm_up(run_steps, warmup, floor_s=None, reset=None):
    """Run `warmup` steps, then more until `floor_s` seconds (default WARMUP_FLOOR_S) of
    stepping have passed, so the clocks and caches have settled before the first timed
    repetition.  reset() (if given) runs after every chunk: the state then never moves more
    than one chunk of steps away from its initial value (a long warm-up on a small mesh
    would otherwise integrate far beyond the configured run)."""
    import torch
    floor_s = WARMUP_FLOOR_S if floor_s is None else floor_s
    t0 = time.perf_counter()
    run_steps(max(warmup, 1))
    torch.cuda.synchronize()
    chunk = max(warmup, 10)
    while time.perf_counter() - t0 < floor_s:
        if reset is not None:
            reset()
        run_steps(chunk)
        torch.cuda.synchronize()
    if reset is not None:
        reset()
    return time.perf_counter() - t0


def timed_reps(run_steps, steps, reps=REPS):
    """Seconds of each of `reps` repetitions of exactly `steps` steps, each bracketed by a
    device synchronisation on both sides."""
    import torch
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_steps(steps)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return out


def time_steps(solver, u, steps, warmup, reps=REPS, t=None, floor_s=None):
    """Warm-up, then `reps` timed repetitions of `steps` RK steps on the product path (one
    dgx_step call per repetition: step pairs replayed from the handle's captured graph).
    The warm-up runs on u itself (the graph is captured for that pointer) and u (and t) are
    restored after every warm-up chunk, so the timed steps start from the configured initial
    state.
    Returns (min seconds, median seconds, warm-up seconds)."""
    run = lambda n: solver.step(u, n, cfl=0.5, t=t)
    u0 = u.clone()
    t0 = None if t is None else t.clone()

    def reset():
        u.copy_(u0)
        if t is not None:
            t.copy_(t0)

    w = warm_up(run, warmup, floor_s, reset)
    if solver.check():
        raise RuntimeError("non-physical state during the warm-up")
    del u0
    secs = timed_reps(run, steps, reps)
    if solver.check():
        raise RuntimeError("non-physical state during the benchmark")
    return min(secs), statistics.median(secs), w


def profiled_stage(solver, u, steps, t=None):
    """The stage kernel's average launch duration (ms), measured with HIP events on the
    handle's stream in a separate pass of `steps` steps (eager launches: the event pairs
    bracket the five stage launches of each step), its launch count and name."""
    import torch
    solver.profile_enable(True)
    solver.step(u, steps, cfl=0.5, t=t)
    torch.cuda.synchronize()
    avg_ms, launches, name = solver.profile_read()
    solver.profile_enable(False)
    if solver.check():
        raise RuntimeError("non-physical state during the benchmark")
    return avg_ms, launches, name


def time_rhs(solver, u, reps, warmup):
    import torch
    du = torch.empty_like(u)
    for _ in range(warmup):
        solver.rhs(u, du)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        solver.rhs(u, du)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def cpu_baseline(cfg, seconds):
    """The oracle as it stands on the host cores, on whole steps of the same workload."""
    import numpy as np

    import oracle
    from paper_2108_06476_amd import inputs
    o = oracle.Oracle(**cfg)
    u = inputs.tgv(o.node_coords())
    nodes = o.num_nodes
    t0 = time.perf_counter()
    steps = 0
    while True:
        u, _ = o.step(u, 1, cfl=0.5)
        steps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    assert np.isfinite(u).all()
    return {"value": steps * 5 * nodes / dt, "unit": "DOF-RHS/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} full RK steps ({5 * steps} RHS) of the same 32^3 N=3 TGV workload, "
                      f"{dt:.1f} s"}


def cpu_baseline_1core(cfg, seconds):
    """The oracle on one host core (the paper's PID study is serial), right-hand sides of the
    same workload."""
    import numpy as np

    import oracle
    from paper_2108_06476_amd import inputs
    o = oracle.Oracle(**cfg)
    u = inputs.tgv(o.node_coords())
    prev = oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        n = 0
        while True:
            du = o.rhs(u)
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(prev)
    assert np.isfinite(du).all()
    return {"value": n * o.num_nodes / dt, "unit": "DOF-RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} right-hand sides of the 32^3 N=3 TGV workload on one core, {dt:.1f} s"}


def bench_rhs_graph(s, u, reps=20, replays=40):
    """The right-hand side alone, reps launches captured once in a HIP graph and replayed."""
    import torch
    du = torch.empty_like(u)
    s.rhs(u, du)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        for _ in range(reps):
            s.rhs(u, du)
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return {"value": reps * replays * s.num_nodes / secs, "unit": "DOF-RHS/s",
            "rhs_per_graph": reps, "replays": replays}


def main():
    global WARMUP_FLOOR_S
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tgv_32")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-measured-peaks", action="store_true",
                    help="skip the HBM copy and FP64 FMA probes (dgx_measure_peak)")
    ap.add_argument("--variants", default="rhs,mixed,batched,sedov,weak,curved,mhd,dwave",
                    help="comma list of extra variants: rhs, mixed, batched, sedov, weak, "
                         "curved, mhd, dwave ('' for none)")
    ap.add_argument("--volume", default=None, help="override the main line's volume integral "
                    "(ec, central, shockcap_hg, weak, weak_mfma)")
    ap.add_argument("--surface", default=None, help="override the main line's surface flux")
    ap.add_argument("--precision", default=None, help="override the main line's precision")
    ap.add_argument("--warmup-floor", type=float, default=WARMUP_FLOOR_S,
                    help="seconds of warm-up at least (0 under a profiler)")
    ap.add_argument("--ensemble-shape", default=None, metavar="BLOCK,GRID",
                    help="fix the ensemble's tile instead of tuning it (e.g. 512,0)")
    ap.add_argument("--rhs-only", action="store_true",
                    help="profiling: time --steps right-hand-side evaluations (dgx_rhs) of the "
                         "main line's configuration instead of RK steps, and stop there (for "
                         "volume-only or surface-only configurations, which may not step)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: every box in this setup has one MI355X, and the "
              "multi-GPU path (element slabs with halo exchange) is a design only. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2108_06476_amd import dgx, inputs
    torch.cuda.set_device(0)
    WARMUP_FLOOR_S = args.warmup_floor
    cfg = dict(inputs.workload(args.workload))
    for key in ("volume", "surface", "precision"):
        if getattr(args, key) is not None:
            cfg[key] = getattr(args, key)
    s = dgx.Solver(**cfg)
    u = make_state(s, args.workload)
    nodes = s.num_nodes
    pkey = profile_key(args.workload, cfg)
    _log(f"workload {args.workload} ({pkey}): E={s.E} nodes={nodes}")
    if args.rhs_only:
        secs = min(time_rhs(s, u, args.steps, args.warmup) for _ in range(3))
        print(json.dumps({"metric": "DOF-RHS evals/sec, right-hand side only (profiling)",
                          "value": args.steps * nodes / secs, "unit": "DOF-RHS/s",
                          "config": {"workload": describe(args.workload, cfg)},
                          "rhs_per_rep": args.steps, "best_of": 3}), flush=True)
        return

    secs, secs_med, warm_s = time_steps(s, u, args.steps, args.warmup)
    value = args.steps * 5 * nodes / secs
    # the stage kernel's average launch duration, from HIP events in a separate pass
    prof_steps = max(args.steps, 20)
    avg_ms, launches, kname = profiled_stage(s, u, prof_steps)
    # dominant kernel: fused volume + surface + lift + Jacobian + RK stage update.
    # Algorithmic bytes per node, averaged over the five stages of a step: each stage reads
    # u and writes u; stages 1-4 write k, stages 2-5 read it (the first stage forms k = dt R,
    # after the last k is dead), so the five stages move 3 + 4 + 4 + 4 + 3 = 18 arrays of 5
    # float64 = 720 B, 144 B per launch.
    alg_bytes = 144.0 * nodes
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(pkey),
                "kernel": kname, "avg_ms": avg_ms, "launches": launches,
                "timing": f"HIP events on the handle's stream, {prof_steps} profiled steps "
                          f"after the timed repetitions",
                "alg_bytes_per_launch": alg_bytes}
    valu = valu_object(stored_pmc(pkey), avg_ms)
    # the board's own peaks beside the published ones (the roofline divides by the latter)
    measured = None if args.no_measured_peaks else measured_peaks(dgx)
    if measured and "error" not in measured:
        roofline["measured_peak"] = measured["hbm_copy_GBs"]
        roofline["frac_of_measured"] = round(achieved / measured["hbm_copy_GBs"], 4)
        if valu:
            valu["measured_peak"] = measured["fp64_fma_TFLOPs"]
            valu["frac_of_measured"] = round(valu["achieved"] / measured["fp64_fma_TFLOPs"], 4)
    _log(f"step: {secs / args.steps * 1e3:.4f} ms/step (min of {REPS}; median "
         f"{secs_med / args.steps * 1e3:.4f}), {value:.4e} DOF-RHS/s; {kname} avg "
         f"{avg_ms * 1e3:.2f} us over {launches} launches")

    out = {"metric": METRIC, "value": value, "unit": "DOF-RHS/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": secs / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "repetitions": REPS, "value_median": args.steps * 5 * nodes / secs_med,
           "ms_per_step_median": secs_med / args.steps * 1e3, "warmup_s": round(warm_s, 3),
           "vs_baseline": None, "dtype": "f64" if cfg.get("precision", "fp64") == "fp64" else "f64+f32",
           "data": "synthetic",
           "config": {"workload": describe(args.workload, cfg),
                      "elements": s.E, "polydeg": 3, "dof_per_var": nodes,
                      "parallelism": "single GPU"},
           "pid_s": 1.0 / value, "roofline": roofline, "valu_fp64": valu,
           "measured_peaks": measured,
           # unique two-point volume fluxes per node and RHS: 3N/2 in 3D (4.5 at N = 3)
           "unique_flux_evals_per_s": value * 1.5 * cfg["polydeg"]}

    variants = {}
    want = [v for v in args.variants.split(",") if v]
    if "rhs" in want:
        try:
            reps = max(20, args.steps)
            t = min(time_rhs(s, u, reps, 5) for _ in range(3))
            variants["rhs_only_fp64"] = {"value": reps * nodes / t, "unit": "DOF-RHS/s",
                                         "rhs_per_rep": reps, "best_of": 3}
        except Exception as e:  # a failing variant must not hide the main line
            variants["rhs_only_fp64"] = {"error": str(e)}
        try:
            variants["rhs_only_fp64_hipgraph"] = bench_rhs_graph(s, u)
        except Exception as e:
            variants["rhs_only_fp64_hipgraph"] = {"error": str(e)}
    if "mixed" in want:
        try:
            for name in ("tgv_32", "tgv_64_mixed", "tgv_n7_32_mixed"):
                c = dict(inputs.workload(name))
                c["precision"] = "mixed"
                sm = dgx.Solver(**c)
                um = make_state(sm, name)
                st = max(6, args.steps // (8 if "64" in name or "n7" in name else 1))
                tm, tmed, _ = time_steps(sm, um, st, 2, reps=3)
                variants[f"mixed_{name}"] = {"value": st * 5 * sm.num_nodes / tm,
                                             "value_median": st * 5 * sm.num_nodes / tmed,
                                             "unit": "DOF-RHS/s", "steps": st, "best_of": 3}
                del sm, um
        except Exception as e:
            variants["mixed"] = {"error": str(e)}
    if "batched" in want:
        for prec in ("fp64", "mixed"):
            try:
                variants[f"batched_{prec}"] = bench_batched(args, prec)
            except Exception as e:
                variants[f"batched_{prec}"] = {"error": str(e)}
    if "sedov" in want:
        try:
            variants["shockcap_sedov_32_fp64"] = bench_sedov(args)
        except Exception as e:
            variants["shockcap_sedov_32_fp64"] = {"error": str(e)}
    if "weak" in want:
        for vol in ("weak", "weak_mfma"):
            try:
                variants[f"{vol}_hll_tgv_32_fp64"] = bench_weak(args, vol)
            except Exception as e:
                variants[f"{vol}_hll_tgv_32_fp64"] = {"error": str(e)}
    if "curved" in want:
        for name in ("curved_4", "curved_32"):
            try:
                variants[f"{name}_mms_fp64"] = bench_curved(args, name)
            except Exception as e:
                variants[f"{name}_mms_fp64"] = {"error": str(e)}
    if "mhd" in want:
        for name in ("alfven_4", "alfven_32"):
            for vol, tag in (("weak", "weak_hll"), ("ec", "ec_ec")):
                try:
                    variants[f"mhd_{name}_{tag}_fp64"] = bench_mhd(args, name, vol)
                except Exception as e:
                    variants[f"mhd_{name}_{tag}_fp64"] = {"error": str(e)}
    if "dwave" in want:
        try:
            variants["density_wave_2d_fp64"] = bench_density_wave(args)
        except Exception as e:
            variants["density_wave_2d_fp64"] = {"error": str(e)}
    out["variants"] = variants

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
        out["cpu_baseline_1core"] = cpu_baseline_1core(cfg, max(4.0, args.cpu_seconds / 2))
    print(json.dumps(out), flush=True)


def bench_batched(args, precision="fp64"):
    """256 independent TGV runs (K in {8,12,16,24}^3, N in {3,4,5}) advanced together: one
    launch per RK stage over all runs, steps replayed from a hipGraph, tile shape autotuned."""
    import torch

    from paper_2108_06476_amd import dgx, inputs
    runs = inputs.ensemble(256, seed=2109)
    cfgs = [dict(inputs.ensemble_config(r), precision=precision) for r in runs]
    b = dgx.Batch(cfgs)
    us, total = [], 0
    for r, c in zip(runs, cfgs):
        o = dgx.Solver(**dict(c, precision="fp64"))
        us.append(inputs.ensemble_state(r, o.node_coords()).contiguous())   # on the GPU
        total += o.num_nodes
        o.close()
    t0 = time.perf_counter()
    if args.ensemble_shape:   # fixed tile (counter runs compare one kernel across passes)
        shape = b.set_shape(*(int(v) for v in args.ensemble_shape.split(",")))
    else:
        shape = b.tune(us, budget_ms=3000)
    tune_s = time.perf_counter() - t0
    run = lambda n: b.step(us, n, cfl=0.5)
    warm_up(run, 2)
    steps = max(4, (args.steps // 20) // 2 * 2)
    secs = timed_reps(run, steps, 3)
    if b.check():
        raise RuntimeError("non-physical state in the ensemble")
    b.close()
    del us
    single = single_run_reference(runs, precision)
    value = steps * 5 * total / min(secs)
    return {"value": value, "unit": "DOF-RHS/s", "runs": len(runs),
            "value_median": steps * 5 * total / statistics.median(secs), "best_of": 3,
            "dof_per_var": total, "steps": steps, "precision": precision,
            "tile_threads": shape[0], "grid_blocks": shape[1], "tune_s": round(tune_s, 2),
            "single_run_node_weighted": single, "vs_single_runs": round(value / single["value"], 4)}


def single_run_reference(runs, precision, steps=4):
    """The ensemble's work done run by run: each (K, N) pair of the ensemble timed as one
    single-run dgx_step (best of 3 after a short warm-up), combined with the ensemble's node
    counts: value = total nodes / sum over pairs of (nodes of the pair / single-run rate)."""
    from paper_2108_06476_amd import dgx, inputs
    pairs = {}
    for r in runs:
        pairs.setdefault((r["K"], r["N"]), []).append(r)
    total, secs_per_rhs = 0, 0.0
    rates = {}
    for (K, N), rs in sorted(pairs.items()):
        c = dict(inputs.ensemble_config(rs[0]), precision=precision)
        s = dgx.Solver(**c)
        u = inputs.ensemble_state(rs[0], s.node_coords()).contiguous()
        tmin, _, _ = time_steps(s, u, steps, 2, reps=3, floor_s=min(0.2, WARMUP_FLOOR_S))
        rate = steps * 5 * s.num_nodes / tmin
        rates[f"K{K}_N{N}"] = round(rate / 1e9, 3)
        nodes = s.num_nodes * len(rs)
        total += nodes
        secs_per_rhs += nodes / rate
        s.close()
    return {"value": total / secs_per_rhs, "unit": "DOF-RHS/s",
            "rate_e9_by_pair": rates, "steps": steps}


def bench_sedov(args):
    """Shock capturing: Sedov blast 32^3, N = 3, HG indicator + blended FV, full RK steps."""
    from paper_2108_06476_amd import dgx, inputs
    s = dgx.Solver(**inputs.workload("sedov_32"))
    u = make_state(s, "sedov_32")
    steps = max(10, args.steps // 10)
    secs, secs_med, _ = time_steps(s, u, steps, 2, reps=3)
    avg_ms, _, _ = profiled_stage(s, u, steps)
    return {"value": steps * 5 * s.num_nodes / secs, "value_median": steps * 5 * s.num_nodes / secs_med,
            "unit": "DOF-RHS/s", "steps": steps, "best_of": 3, "stage_us": round(avg_ms * 1e3, 2)}


def bench_density_wave(args):
    """2D density wave 16^2, N = 3: 100 RK steps (launch-bound at this size)."""
    import torch

    from paper_2108_06476_amd import dgx, inputs
    s = dgx.Solver(**inputs.workload("density_wave_2d"))
    u = make_state(s, "density_wave_2d")
    secs, _, _ = time_steps(s, u, 100, 5, reps=3)
    del torch
    return {"value": 100 * 5 * s.num_nodes / secs, "unit": "DOF-RHS/s", "steps": 100,
            "ms_per_step": secs / 100 * 1e3, "best_of": 3}


def bench_weak(args, volume="weak"):
    """Weak-form DG + HLL on the 32^3 N = 3 TGV (the paper's other measured solver), with the
    line contractions on the VALU ("weak") or on the matrix cores ("weak_mfma"): full RK
    steps, with the stage kernel's live average and its HBM fraction (same 144 B/node)."""
    from paper_2108_06476_amd import dgx, inputs
    cfg = dict(inputs.workload("tgv_32"), volume=volume, surface="hll")
    s = dgx.Solver(**cfg)
    u = make_state(s, "tgv_32")
    steps = max(10, args.steps // 2)
    secs, secs_med, _ = time_steps(s, u, steps, 2, reps=3)
    avg_ms, _, _ = profiled_stage(s, u, steps)
    gbs = 144.0 * s.num_nodes / (avg_ms * 1e-3) / 1e9
    return {"value": steps * 5 * s.num_nodes / secs, "value_median": steps * 5 * s.num_nodes / secs_med,
            "unit": "DOF-RHS/s", "steps": steps, "best_of": 3,
            "stage_us": round(avg_ms * 1e3, 2), "stage_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def bench_curved(args, name):
    """The PID study's curvilinear mesh (warped box, Eq. (2)) with the manufactured solution's
    source term, EC + LLF, N = 3: full RK steps; curved_4 is the paper's 4^3 mesh (4096
    nodes: launch-bound), curved_32 the same per-GPU size as tgv_32."""
    import torch

    from paper_2108_06476_amd import dgx, inputs
    s = dgx.CurvSolver(**inputs.workload(name))
    u = inputs.mms(s.node_coords()).contiguous()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    steps = max(10, args.steps // 2)
    secs, secs_med, _ = time_steps(s, u, steps, 2, reps=3, t=t)
    out = {"value": steps * 5 * s.num_nodes / secs, "unit": "DOF-RHS/s", "steps": steps,
           "value_median": steps * 5 * s.num_nodes / secs_med, "best_of": 3,
           "ms_per_step": secs / steps * 1e3}
    if not name.endswith("_4"):   # the 4^3 mesh: its launches are latency chains
        out["stage_us"] = round(profiled_stage(s, u, steps, t=t)[0] * 1e3, 2)
    return out


def bench_mhd(args, name, volume="weak"):
    """Ideal MHD, N = 3, on the Alfven wave: weak form + HLL, or EC flux differencing with
    Powell's term and EC surfaces; the paper's 4^3 mesh (launch-bound) and 32^3 (the
    per-GPU size of tgv_32); full RK steps."""
    import torch

    from paper_2108_06476_amd import dgx, inputs
    cfg = dict(inputs.workload(name))
    if volume == "ec":
        cfg.update(volume="ec", surface="ec")
    s = dgx.MhdSolver(**cfg)
    u = inputs.alfven(s.node_coords()).contiguous()
    steps = max(10, args.steps // 2)
    secs, secs_med, _ = time_steps(s, u, steps, 2, reps=3)
    out = {"value": steps * 5 * s.num_nodes / secs, "unit": "DOF-RHS/s", "steps": steps,
           "value_median": steps * 5 * s.num_nodes / secs_med, "best_of": 3,
           "ms_per_step": secs / steps * 1e3}
    if not name.endswith("_4"):   # the 4^3 mesh: its launches are latency chains
        avg_ms = profiled_stage(s, u, steps)[0]
        # stage traffic: 8 variables, 18 arrays per step over 5 stages (as for Euler)
        gbs = 8 * 8 * 3.6 * s.num_nodes / (avg_ms * 1e-3) / 1e9
        out.update(stage_us=round(avg_ms * 1e3, 2), stage_hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
    return out


WORKLOAD_TEXT = {
    "tgv_32": "3D Euler Taylor-Green vortex Mach 0.1 + 1% seeded density perturbation, DGSEM "
              "N=3, 32^3 periodic hex elements on [-pi,pi]^3",
    "sedov_32": "3D Euler Sedov-type Gaussian blast (width 0.25), DGSEM N=3, 32^3 periodic hex "
                "elements on [-1,1]^3, Hennemann-Gassner indicator (alpha_max 0.5) with blended "
                "DG/FV subcell volume",
    "tgv_64_mixed": "3D Euler Taylor-Green vortex Mach 0.1, DGSEM N=3, 64^3 hex elements",
    "tgv_n7_32_mixed": "3D Euler Taylor-Green vortex Mach 0.1, DGSEM N=7, 32^3 hex elements",
    "density_wave_2d": "2D Euler density wave, DGSEM N=3, 16^2 periodic quads on [-2,2]^2",
}


def describe(workload, cfg):
    """The workload of the main line in words (configuration overrides included)."""
    return (f"{workload}: {WORKLOAD_TEXT.get(workload, workload)}; volume {cfg['volume']}, "
            f"surface {cfg['surface']}, {cfg.get('precision', 'fp64')}, CK(5,4) RK at CFL 0.5")


def profile_key(workload, cfg):
    """Name of the committed counter summary that applies to the main line's stage kernel:
    k_stage_<workload>_<precision> for the workload's own scheme, with the volume and surface
    appended when they were overridden."""
    from paper_2108_06476_amd import inputs
    base = inputs.workload(workload)
    key = "k_stage_" + workload.replace("_", "") + "_" + cfg.get("precision", "fp64")
    if cfg["volume"] != base["volume"] or cfg["surface"] != base["surface"]:
        key += f"_{cfg['volume']}_{cfg['surface']}"
    return key


def kernel_source_hash():
    """Hash of the HIP sources; a stored counter measurement applies only to this build."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2108_06476_amd", "csrc", "*"))):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(os.path.basename(f).encode())
            h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_peaks(dgx):
    """dgx_measure_peak on this board: the copy bandwidth of a 2 GiB float64 buffer (GB/s,
    read + written) and the FP64 vector FMA rate (TFLOP/s), each the best of 10 launches."""
    try:
        out = {k: round(dgx.measure_peak(k), 2) for k in ("hbm_copy_GBs", "fp64_fma_TFLOPs")}
    except Exception as e:  # a failing probe must not hide the main line
        return {"error": str(e)}
    out["method"] = ("dgx_measure_peak: a grid-stride copy of 2 GiB (four 16-byte non-temporal loads in flight per lane), and "
                     "eight independent FP64 FMA chains per lane at 8 waves per SIMD; best of 10")
    _log(f"measured peaks: HBM copy {out['hbm_copy_GBs']:.0f} GB/s, FP64 FMA "
         f"{out['fp64_fma_TFLOPs']:.1f} TFLOP/s")
    return out


def valu_object(pmc, avg_ms):
    """The stage kernel against the FP64 vector peak: FP64 flops per launch from the committed
    counter summary (64 lanes x (ADD + MUL + TRANS + 2 FMA) FP64 VALU instructions, masked
    lanes included) over the live launch time avg_ms, and all its vector instructions against
    the issue peak; None without a summary of the current sources."""
    if pmc is None or not pmc.get("fp64_flops_per_launch"):
        return None
    tf = pmc["fp64_flops_per_launch"] / (avg_ms * 1e-3) / 1e12
    valu = {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tf / FP64_VALU_PEAK_TFLOPS, 4),
            "fp64_flops_per_launch": pmc["fp64_flops_per_launch"],
            "valu_insts_per_wave": pmc.get("valu_insts_per_wave"),
            "fp64_share_of_valu_insts": pmc.get("fp64_share_of_valu_insts")}
    cpl = pmc.get("counters_per_launch", {})
    if cpl.get("SQ_INSTS_VALU"):
        # all vector instructions (float64, address, select, move) against the issue peak
        rate = cpl["SQ_INSTS_VALU"] / (avg_ms * 1e-3)
        valu["issue"] = {"achieved": round(rate / 1e9, 1), "peak": round(VALU_ISSUE_PEAK / 1e9, 1),
                         "unit": "G wave-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4)}
    return valu


def stored_pmc(name):
    """The committed counter summary of `name`, or None when it is missing or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{name}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec


def stored_traffic(name):
    """HBM bytes per launch of `name` from the committed counter summary (None as above)."""
    rec = stored_pmc(name)
    return None if rec is None else rec.get("traffic_bytes_per_launch")


if __name__ == "__main__":
    main()
