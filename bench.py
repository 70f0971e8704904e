#!/usr/bin/env python3
"""Throughput of the batched physics step on one MI355X.

Workload: humanoid-like robot (13 capsule bodies, free root + 21 revolute DOFs), 4096 envs,
dt = 1/60 s with 2 substeps, 8 PGS sweeps, seeded actions U[-1, 1] x 67.5, ground contact on every
body, starting from the seeded standing pose.  One step = one env-step of every env (both substeps).

Prints one JSON line.  `value` is env-steps/s of the step that meets the stated tolerance against
the FP64 oracle (FP64 compute, FP32 tensors); the FP32-compute step is reported beside it.
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

METRIC = "env-steps/s fwd and fwd+bwd, 4096-env humanoid, at stated err vs FP64 oracle"

# algorithmic cost per env-step of the humanoid workload (two substeps), R = mean constraint rows per
# substep: flops ~ 37e3 + 5.1e3 R; bytes = state + actions read, state + contact forces written
FLOPS_BASE, FLOPS_PER_ROW = 37.0e3, 5.1e3
BYTES_PER_ENV_STEP = 680.0
PEAK_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP32 unpacked == FP64 vector)
PEAK_HBM_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "step_kernel_humanoid4096.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2108_10470_amd", "csrc", f) for f in ("ags_step.hip", "ags_internal.h")]


def measured_traffic(variant):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    try:
        with open(PROFILE) as fh:
            line = next(l for l in fh if l.startswith("traffic_bytes_per_launch"))
    except (OSError, StopIteration):
        return None
    kv = dict(t.split("=") for t in line.split()[1:])
    if kv.get("source") != h.hexdigest()[:16] or variant not in kv:
        return None
    return float(kv[variant])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--precision", choices=["both", "fp64", "fp32"], default="both")
    ap.add_argument("--cpu-envs", type=int, default=4096, help="oracle sample: envs")
    ap.add_argument("--cpu-steps", type=int, default=600, help="oracle sample: steps from the seeded start")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the replay that measures mean active rows")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (scale reference for HBM counters)")
    return ap.parse_args()


def run_gpu(env, params, n_envs, steps, warmup, fp64, actions_dev, root0, dof0):
    import torch
    from paper_2108_10470_amd import ags
    model = ags.Model(env)
    sim = ags.Sim([model], [0] * n_envs, params, device="cuda:0", fp64=fp64)
    sim.root_state.copy_(root0)
    sim.dof_state.copy_(dof0)
    stream = torch.cuda.current_stream()
    nd = env.n_dof
    for t in range(warmup):
        sim.bind(ags.DOF_ACTUATION, actions_dev[t])
        sim.step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for t in range(steps):
        sim.bind(ags.DOF_ACTUATION, actions_dev[warmup + t])
        ev[t][0].record(stream)
        sim.step()
        ev[t][1].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    launch_ms = np.array([a.elapsed_time(b) for a, b in ev])
    finite = bool(torch.isfinite(sim.root_state).all() and torch.isfinite(sim.dof_state).all())
    return dict(total_ms=total_ms, wall_s=wall, launch_ms=launch_ms, finite=finite)


def mean_rows(env, params, n_envs, steps, fp64, actions_dev, root0, dof0):
    """Replays the same (deterministic) run with the row-count output bound."""
    import torch
    from paper_2108_10470_amd import ags
    model = ags.Model(env)
    sim = ags.Sim([model], [0] * n_envs, params, device="cuda:0", fp64=fp64, debug=True)
    sim.root_state.copy_(root0)
    sim.dof_state.copy_(dof0)
    acc = torch.zeros((), dtype=torch.float64, device="cuda:0")
    for t in range(steps):
        sim.bind(ags.DOF_ACTUATION, actions_dev[t])
        sim.step()
        acc += sim.dbg_rc.double().mean()
    torch.cuda.synchronize()
    return float(acc.item() / steps)


def cpu_baseline(env, params, n_envs, n_steps):
    """The FP64 oracle on the host cores over a bounded sample of the same workload."""
    from oracle import oracle as O
    from paper_2108_10470_amd import workloads as W
    threads = max(1, min(16, os.cpu_count() or 1))
    oe = O.OracleEnv(env)
    root, dof = W.initial_state(env, n_envs, 0)
    acts = W.actuation(env, n_envs, n_steps, 0)
    t0 = time.perf_counter()
    for t in range(n_steps):
        o = oe.step(params, root, dof, acts[t], n_threads=threads)
        root, dof = o["root"], o["dof"]
    dt = time.perf_counter() - t0
    return {"value": n_envs * n_steps / dt, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_envs} humanoid envs x {n_steps} env-steps from the seeded standing start "
                      f"(standing, falling, lying), FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the step has no cross-GPU work "
              f"and this build measures the single-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2108_10470_amd import workloads as W
    env = W.env_humanoid()
    params = W.SimParams()
    E, K, Wm = args.envs, args.steps, args.warmup
    root, dof = W.initial_state(env, E, 0)
    acts = W.actuation(env, E, Wm + K, 0).astype(np.float32)
    actions_dev = torch.from_numpy(acts).to("cuda:0").reshape(Wm + K, -1)
    actions_dev = [actions_dev[t] for t in range(Wm + K)]
    root0 = torch.from_numpy(root.reshape(-1, 13).astype(np.float32)).to("cuda:0")
    dof0 = torch.from_numpy(dof.reshape(-1, 2).astype(np.float32)).to("cuda:0")
    print(f"[bench] humanoid envs={E} steps={K} warmup={Wm}", file=sys.stderr, flush=True)
    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    variants = {"both": [True, False], "fp64": [True], "fp32": [False]}[args.precision]
    res = {}
    for fp64 in variants:
        name = "fp64" if fp64 else "fp32"
        r = run_gpu(env, params, E, K, Wm, fp64, actions_dev, root0, dof0)
        r["rows"] = None if args.no_rows else mean_rows(env, params, E, Wm + K, fp64, actions_dev, root0, dof0)
        res[name] = r
        print(f"[bench] {name}: {K} steps in {r['total_ms']:.1f} ms, launch mean {r['launch_ms'].mean():.3f} ms, "
              f"rows/substep {r['rows']}, finite {r['finite']}", file=sys.stderr, flush=True)

    head = "fp64" if "fp64" in res else "fp32"
    h = res[head]
    value = E * K / (h["total_ms"] / 1e3)
    t_launch = float(h["launch_ms"].mean()) / 1e3
    rows = h["rows"] if h["rows"] is not None else float("nan")
    flops = E * (FLOPS_BASE + FLOPS_PER_ROW * rows)
    ach_tf = flops / t_launch / 1e12
    ach_gbs = E * BYTES_PER_ENV_STEP / t_launch / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": h["total_ms"] / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": "humanoid-like, 4096 envs (13 capsules, free root + 21 revolute DOFs), "
                               "dt 1/60 s x 2 substeps, 8 PGS sweeps, actions U[-1,1] x 67.5",
                   "envs": E, "substeps": params.substeps, "pgs_iters": params.pgs_iters,
                   "tensors": "f32", "compute": head, "mean_rows_per_substep": rows},
        "roofline": {"bound": "alu", "achieved": ach_tf, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach_tf / PEAK_VALU_TFLOPS, "traffic": measured_traffic(head),
                     "kernel": "step_kernel<double>" if head == "fp64" else "step_kernel<float>",
                     "launch_ms": t_launch * 1e3,
                     "hbm": {"achieved": ach_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach_gbs / PEAK_HBM_GBS,
                             "bytes_per_env_step": BYTES_PER_ENV_STEP},
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"},
        "fwd_bwd": None,
        "variants": {k: {"env_steps_per_s": E * K / (v["total_ms"] / 1e3), "ms_per_step": v["total_ms"] / K,
                         "launch_ms": float(v["launch_ms"].mean()), "mean_rows_per_substep": v["rows"],
                         "finite": v["finite"]} for k, v in res.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W.env_humanoid(), params, args.cpu_envs, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
