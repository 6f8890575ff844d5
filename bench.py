#!/usr/bin/env python3
"""Benchmark: DOF-RHS evaluations per second of the DGSEM Euler step on one MI355X.

Workload (default): 3D compressible Euler, Taylor-Green vortex at Mach 0.1 with a seeded 1 %
smooth density perturbation, DGSEM N = 3 on 32^3 periodic hex elements ([-pi, pi]^3), EC
flux-differencing volume integral + LLF surface flux, Carpenter-Kennedy 5-stage RK with the
CFL 0.5 time step, float64.  A timed step is one full RK step (time step + 5 stages of
interface fluxes and volume/lift/Jacobian/stage update), inputs resident in HBM.

value = steps * 5 * E * (N+1)^3 / seconds (the paper's PID, Eq. (3), is 1/value).
Also reported: the right-hand side alone, the mixed-precision and the ensemble variants,
the roofline of the dominant kernel (live HIP-event timing) and the oracle on the host.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-RHS evals/sec (PID) 3D Euler N=3, FP64 vs mixed vs batched, 1 MI355X"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_state(solver, name):
    import torch

    from paper_2108_06476_amd import inputs
    xyz = solver.node_coords().cpu().numpy()
    if name.startswith("tgv"):
        u = inputs.tgv(xyz)
    elif name.startswith("sedov"):
        u = inputs.sedov(xyz)
    else:
        u = inputs.density_wave(xyz)
    return torch.from_numpy(u).cuda()


def time_steps(solver, u, steps, warmup, profile=False):
    import torch
    solver.step(u, warmup, cfl=0.5)
    torch.cuda.synchronize()
    if profile:
        solver.profile_enable(True)
    t0 = time.perf_counter()
    solver.step(u, steps, cfl=0.5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = solver.profile_read() if profile else None
    if profile:
        solver.profile_enable(False)
    if solver.check():
        raise RuntimeError("non-physical state during the benchmark")
    return t1 - t0, prof


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tgv_32")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="rhs,mixed,batched",
                    help="comma list of extra variants: rhs, mixed, batched ('' for none)")
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
    cfg = inputs.workload(args.workload)
    s = dgx.Solver(**cfg)
    u = make_state(s, args.workload)
    nodes = s.num_nodes
    _log(f"workload {args.workload}: E={s.E} nodes={nodes}")

    secs, prof = time_steps(s, u, args.steps, args.warmup, profile=True)
    value = args.steps * 5 * nodes / secs
    avg_ms, launches, kname = prof
    # dominant kernel: fused volume + lift + Jacobian + RK stage update.  Algorithmic bytes
    # per node and stage: read u and k, write k and u (4 x 5 float64 = 160 B).
    alg_bytes = 160.0 * nodes
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": kname, "avg_ms": avg_ms, "launches": launches}
    _log(f"step: {secs / args.steps * 1e3:.3f} ms/step, {value:.4e} DOF-RHS/s; "
         f"{kname} avg {avg_ms * 1e3:.1f} us")

    out = {"metric": METRIC, "value": value, "unit": "DOF-RHS/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": secs / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "tgv_32: 3D Euler Taylor-Green vortex Mach 0.1 + 1% seeded "
                                  "density perturbation, DGSEM N=3, 32^3 periodic hex elements on "
                                  "[-pi,pi]^3, EC volume + LLF surface, CK(5,4) RK at CFL 0.5",
                      "elements": s.E, "polydeg": 3, "dof_per_var": nodes,
                      "parallelism": "single GPU"},
           "pid_s": 1.0 / value, "roofline": roofline}

    variants = {}
    want = [v for v in args.variants.split(",") if v]
    if "rhs" in want:
        try:
            reps = max(20, args.steps)
            t = time_rhs(s, u, reps, 5)
            variants["rhs_only_fp64"] = {"value": reps * nodes / t, "unit": "DOF-RHS/s"}
        except Exception as e:  # a failing variant must not hide the main line
            variants["rhs_only_fp64"] = {"error": str(e)}
    if "mixed" in want:
        try:
            for name in ("tgv_32", "tgv_64_mixed", "tgv_n7_32_mixed"):
                c = dict(inputs.workload(name))
                c["precision"] = "mixed"
                sm = dgx.Solver(**c)
                um = make_state(sm, name)
                st = max(5, args.steps // (8 if "64" in name or "n7" in name else 1))
                tm, _ = time_steps(sm, um, st, 2)
                variants[f"mixed_{name}"] = {"value": st * 5 * sm.num_nodes / tm,
                                             "unit": "DOF-RHS/s", "steps": st}
                del sm, um
        except Exception as e:
            variants["mixed"] = {"error": str(e)}
    if "batched" in want:
        try:
            variants["batched_fp64"] = bench_batched(args)
        except Exception as e:
            variants["batched_fp64"] = {"error": str(e)}
    out["variants"] = variants

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """256 independent TGV runs (K in {8,12,16,24}^3, N in {3,4,5}) advanced together."""
    import ctypes as C

    import torch

    from paper_2108_06476_amd import dgx, inputs
    runs = inputs.ensemble(256, seed=2109)
    cfgs = (dgx.Config * len(runs))(*[dgx.make_config(**inputs.ensemble_config(r)) for r in runs])
    L = dgx.lib()
    b = C.c_void_p()
    st = L.dgx_batch_create(cfgs, len(runs), C.c_void_p(torch.cuda.current_stream().cuda_stream),
                            C.byref(b))
    if st != 0:
        raise RuntimeError(f"dgx_batch_create failed: {st}")
    try:
        us, total = [], 0
        for r in runs:
            c = inputs.ensemble_config(r)
            o = dgx.Solver(**c)
            xyz = o.node_coords().cpu().numpy()
            us.append(torch.from_numpy(inputs.ensemble_state(r, xyz)).cuda())
            total += o.num_nodes
            o.close()
        ptrs = (C.c_void_p * len(us))(*[C.c_void_p(t.data_ptr()) for t in us])
        steps = max(3, args.steps // 40)
        st = L.dgx_batch_step(b, ptrs, 1, C.c_double(0.5), None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st |= L.dgx_batch_step(b, ptrs, steps, C.c_double(0.5), None)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        if st != 0:
            raise RuntimeError(L.dgx_batch_last_error(b).decode())
        return {"value": steps * 5 * total / secs, "unit": "DOF-RHS/s", "runs": len(runs),
                "dof_per_var": total, "steps": steps}
    finally:
        L.dgx_batch_destroy(b)


if __name__ == "__main__":
    main()
