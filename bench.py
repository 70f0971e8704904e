#!/usr/bin/env python3
"""Throughput of the batched physics step on one MI355X.

Workload: humanoid-like robot (13 capsule bodies, free root + 21 revolute DOFs), 4096 envs,
dt = 1/60 s with 2 substeps, 8 PGS sweeps, seeded actions U[-1, 1] x 67.5, ground contact on every
body.  With random actions and no resets the humanoids fall within ~60 steps and spend the rest of a
1000-step run on the ground, so every measurement starts from the state an untimed pre-roll of
--preroll steps (default 200, FP32 kernel) reaches from the seeded standing pose: the timed window is
the same regime whatever --steps is.  One step = one env-step of every env (both substeps).

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
# substep: flops ~ 37e3 + 5.1e3 R; bytes = state (55 floats) + actions (21) read, state + the 13 bodies' contact
# forces (39) + the DOF forces (21, an output the bench binds) written
FLOPS_BASE, FLOPS_PER_ROW = 37.0e3, 5.1e3
BYTES_PER_ENV_STEP = 764.0
PEAK_VALU_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP32 unpacked == FP64 vector)
PEAK_HBM_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_2108_10470_amd", "csrc")
PROFILES = {"step": (os.path.join(ROOT, "profiles", "step_kernel_humanoid4096.md"), ("ags_step.hip", "ags_internal.h")),
            "adjoint": (os.path.join(ROOT, "profiles", "adjoint_kernel_humanoid4096.md"),
                        ("ags_adjoint.hip", "ags_internal.h"))}


def measured_traffic(variant, kernel="step"):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    PROFILE, sources = PROFILES[kernel]
    h = hashlib.sha256()
    for f in (os.path.join(CSRC, x) for x in sources):
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
    ap.add_argument("--preroll", type=int, default=200,
                    help="untimed steps (FP32 kernel) from the standing start before every measurement")
    ap.add_argument("--rows-ref-steps", type=int, default=1000,
                    help="length of the run from the standing start whose mean row count is reported beside "
                         "the window's (FP32 kernel; 0 skips it)")
    ap.add_argument("--envs", type=int, default=4096)
    ap.add_argument("--precision", choices=["both", "fp64", "fp32"], default="both")
    ap.add_argument("--cpu-envs", type=int, default=4096, help="oracle sample: envs (all host threads)")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle sample: steps of the timed window")
    ap.add_argument("--cpu-envs-1core", type=int, default=512, help="oracle sample on one thread: envs")
    ap.add_argument("--cpu-steps-1core", type=int, default=10, help="oracle sample on one thread: steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the replay that measures mean active rows")
    ap.add_argument("--no-fwd-bwd", action="store_true", help="skip the forward+adjoint rollout measurement")
    ap.add_argument("--fwd-bwd-steps", type=int, default=64)
    ap.add_argument("--fwd-bwd-every", type=int, default=0,
                    help="checkpoint interval of the headline forward+adjoint rollout; 0 stores the whole tape")
    ap.add_argument("--fwd-bwd-ckpt-every", type=int, default=16,
                    help="checkpoint interval of the secondary (recomputing) forward+adjoint measurement")
    ap.add_argument("--fwd-bwd-reps", type=int, default=3)
    ap.add_argument("--no-hetero", action="store_true", help="skip the heterogeneous-batch measurement")
    ap.add_argument("--no-tgs", action="store_true",
                    help="skip the temporal Gauss-Seidel and randomized-property variants' measurements")
    ap.add_argument("--hetero-envs", type=int, default=16384)
    ap.add_argument("--hetero-steps", type=int, default=100)
    ap.add_argument("--hetero-preroll", type=int, default=100)
    ap.add_argument("--no-ant-grad", action="store_true",
                    help="skip the differentiation workload (4096 ant-like envs, 64-step rollout, checkpoints "
                         "every 16)")
    ap.add_argument("--no-hand", action="store_true", help="skip the 65536-env hand+cube measurement")
    ap.add_argument("--hand-envs", type=int, default=65536)
    ap.add_argument("--hand-steps", type=int, default=32)
    ap.add_argument("--phase-report", action="store_true",
                    help="instead of the benchmark: per-phase shader-clock cycles of the step (FP64, FP32) and of the "
                         "adjoint's dense row responses on the pre-rolled window, one JSON line")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (scale reference for HBM counters)")
    return ap.parse_args()


def preroll(env, params, n_envs, steps, actions_dev, root0, dof0):
    """Untimed steps with the FP32 kernel from the standing start; returns copies of the state reached."""
    import torch
    from paper_2108_10470_amd import ags
    sim = ags.Sim([ags.Model(env)], [0] * n_envs, params, device="cuda:0", fp64=False)
    sim.root_state.copy_(root0)
    sim.dof_state.copy_(dof0)
    for t in range(steps):
        sim.bind(ags.DOF_ACTUATION, actions_dev[t])
        sim.step()
    torch.cuda.synchronize()
    return sim.root_state.clone(), sim.dof_state.clone()


def run_gpu(env, params, n_envs, steps, warmup, fp64, actions_dev, root0, dof0, props=None):
    """warmup untimed steps from (root0, dof0) with actions_dev[0:warmup], then `steps` timed steps with
    the following actions (HIP events around each launch and around the whole window); then the first
    chunk of the same window captured in a HIP graph whose first nodes restore the window's start state,
    replayed, and the same chunk run eagerly from the same state (like-for-like graph vs eager)."""
    import torch
    from paper_2108_10470_amd import ags
    model = ags.Model(env)
    sim = ags.Sim([model], [0] * n_envs, params, device="cuda:0", fp64=fp64)
    if props is not None:  # per-env property tensors (domain randomization)
        t = {k: torch.tensor(v, dtype=torch.float32, device="cuda:0") for k, v in props.items()}
        sim.set_properties(mass_scale=t["mass_scale"].reshape(-1).contiguous(),
                           stiffness=t["stiffness"].reshape(-1).contiguous(),
                           damping=t["damping"].reshape(-1).contiguous(), limits=t["limits"].reshape(-1, 2).contiguous(),
                           friction=t["friction"].contiguous(), gravity=t["gravity"].contiguous())
    sim.root_state.copy_(root0)
    sim.dof_state.copy_(dof0)
    stream = torch.cuda.current_stream()
    for t in range(warmup):
        sim.bind(ags.DOF_ACTUATION, actions_dev[t])
        sim.step()
    torch.cuda.synchronize()
    win_root, win_dof = sim.root_state.clone(), sim.dof_state.clone()
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
    fin_env = (torch.isfinite(sim.root_state).view(n_envs, -1).all(1) & torch.isfinite(sim.dof_state).view(n_envs, -1).all(1))
    finite = bool(fin_env.all())
    finite_frac = float(fin_env.double().mean())
    graph_ms = eager_ms = None
    chunk = min(50, steps)
    if chunk > 0:
        def body():
            sim.root_state.copy_(win_root)
            sim.dof_state.copy_(win_dof)
            for t in range(chunk):
                sim.bind(ags.DOF_ACTUATION, actions_dev[warmup + t])
                sim.step()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        body()  # eager, same steps
        torch.cuda.synchronize()
        a.record(stream)
        body()
        b.record(stream)
        torch.cuda.synchronize()
        eager_ms = a.elapsed_time(b) / chunk
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            body()
        g.replay()
        torch.cuda.synchronize()
        reps = max(1, steps // chunk)
        a.record(stream)
        for _ in range(reps):
            g.replay()
        b.record(stream)
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b) / (reps * chunk)
    return dict(total_ms=total_ms, wall_s=wall, launch_ms=launch_ms, finite=finite, finite_frac=finite_frac, graph_ms=graph_ms,
                eager_same_steps_ms=eager_ms, graph_chunk=chunk, window_root=win_root, window_dof=win_dof)


def mean_rows(env, params, n_envs, steps, fp64, actions_dev, root0, dof0, skip=0):
    """Replays the same (deterministic) run with the row-count output bound: mean rows per env-substep
    over steps [skip, steps)."""
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
        if t >= skip:
            acc += sim.dbg_rc.double().mean()
    torch.cuda.synchronize()
    return float(acc.item() / max(1, steps - skip))


def run_fwd_bwd(env, params, n_envs, fp64, actions, root0, dof0, every, reps, adjoint_precision=0, control=None):
    """Forward rollout of T = len(actions) steps with a checkpoint every `every` steps, then the reverse
    pass (segment recomputation + adjoint of every step) for L = sum of final root x positions; with
    every = 0 the forward pass stores the whole tape and the reverse pass recomputes nothing.  control:
    the per-step control the actions drive (DOF actuation, or PD position targets)."""
    import ctypes
    import torch
    from paper_2108_10470_amd import ags
    control = ags.DOF_ACTUATION if control is None else control
    sim = ags.Sim([ags.Model(env)], [0] * n_envs, params, device="cuda:0", fp64=fp64,
                  adjoint_precision=adjoint_precision, pd=control == ags.DOF_POS_TARGET)
    L = ags.lib()
    T = actions.shape[0]
    n = ctypes.c_int64()
    L.ags_rollout_state_size(sim.h, ctypes.byref(n))
    f32 = dict(dtype=torch.float32, device="cuda:0")
    nb = ctypes.c_int64()
    if every == 0:
        ags._check(L.ags_rollout_tape_bytes(sim.h, T, ctypes.byref(nb)), "rollout_tape_bytes")
        tape = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
        ckpt = tape[:4 * n.value].view(torch.float32).view(1, n.value)  # the state before step 0
    else:
        ckpt = torch.empty(((T + every - 1) // every, n.value), **f32)
        ags._check(L.ags_rollout_seg_bytes(sim.h, every, ctypes.byref(nb)), "rollout_seg_bytes")
        seg = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    root_adj = torch.empty_like(sim.root_state)
    dof_adj = torch.empty_like(sim.dof_state)
    act_adj = torch.empty_like(actions)
    status = torch.zeros(n_envs, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())

    def one():
        sim.root_state.copy_(root0)
        sim.dof_state.copy_(dof0)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        root_adj.zero_()
        root_adj[:, 0] = 1.0
        dof_adj.zero_()
        e0.record(stream)
        if every == 0:
            ags._check(L.ags_rollout_forward_tape(sim.h, T, control, P(actions), P(tape), sp), "rollout_forward_tape")
        else:
            ags._check(L.ags_rollout_forward(sim.h, T, every, control, P(actions), P(ckpt), sp), "rollout_forward")
        e1.record(stream)
        if every == 0:
            ags._check(L.ags_rollout_backward_tape(sim.h, T, control, P(actions), P(tape), P(root_adj), P(dof_adj),
                                                   P(act_adj), P(status), sp), "rollout_backward_tape")
        else:
            ags._check(L.ags_rollout_backward(sim.h, T, every, control, P(actions), P(ckpt), P(seg), P(root_adj),
                                              P(dof_adj), P(act_adj), P(status), sp), "rollout_backward")
        e2.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2)

    one()
    times = [one() for _ in range(reps)]
    fwd = float(np.median([t[0] for t in times]))
    bwd = float(np.median([t[1] for t in times]))
    # gradient summary of the rollout: mean |dL/d action| over everything, and the median over envs of each
    # env's mean (a few envs near a non-smooth contact event can dominate the first)
    g = act_adj.abs().double().reshape(T, n_envs, -1)
    grad_mean = float(g.mean())
    grad_median_env = float(g.mean(dim=(0, 2)).median())
    finite = bool(torch.isfinite(act_adj).all())
    # the adjoint kernel alone: one launch per step on a fixed state (the checkpoint of the first segment),
    # the seed restored before every launch (the call overwrites it with the adjoint of the earlier state)
    x = ckpt[0]
    nr = 13 * sim.shapes[ags.ROOT_STATE][0]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    aa = torch.empty_like(act_adj[0])
    for a, b in evs:
        root_adj.zero_()
        root_adj[:, 0] = 1.0
        dof_adj.zero_()
        a.record(stream)
        L.ags_sim_step_backward(sim.h, P(x), ctypes.c_void_p(x.data_ptr() + 4 * nr), P(actions[0]), P(root_adj),
                                P(dof_adj), P(aa), P(status), sp)
        b.record(stream)
    torch.cuda.synchronize()
    adj_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    return {"value": n_envs * T / ((fwd + bwd) / 1e3), "unit": "env-steps/s", "steps": T,
            "checkpoint_every": every if every else "none: whole tape stored in the forward pass",
            "ms_forward": fwd, "ms_backward": bwd, "adjoint_launch_ms": adj_ms,
            "envs_over_row_capacity": int((status != 0).sum()), "finite": finite,
            "grad_abs_mean": grad_mean, "grad_abs_median_env": grad_median_env, "dtype": "f64" if fp64 else "f32",
            "adjoint_dtype": "f64" if adjoint_precision == 64 or (adjoint_precision == 0 and fp64) else "f32",
            "loss": "sum over envs of the final torso x position", "reps": reps,
            "adjoint_traffic_bytes_per_launch": measured_traffic(
                "fp64" if adjoint_precision == 64 or (adjoint_precision == 0 and fp64) else "fp32", "adjoint")}


def run_jacmass(env, params, n_envs, root0, dof0, reps=20):
    """Jacobian and mass-matrix tensors of the whole batch at the start state (ags_sim_jacobian_mass):
    mean launch time and the output bytes it writes."""
    import torch
    from paper_2108_10470_amd import ags
    sim = ags.Sim([ags.Model(env)], [0] * n_envs, params, device="cuda:0")
    sim.root_state.copy_(root0)
    sim.dof_state.copy_(dof0)
    info = sim.models[0].info
    J = torch.empty((n_envs, info.n_links, 6, info.n_v), dtype=torch.float32, device="cuda:0")
    M = torch.empty((n_envs, info.n_v, info.n_v), dtype=torch.float32, device="cuda:0")
    import ctypes
    L = ags.lib()
    stream = torch.cuda.current_stream()
    call = lambda: ags._check(L.ags_sim_jacobian_mass(sim.h, 0, ctypes.c_void_p(J.data_ptr()),
                                                       ctypes.c_void_p(M.data_ptr()),
                                                       ctypes.c_void_p(stream.cuda_stream)), "jacobian_mass")
    call()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        call()
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    out_bytes = 4 * (J.numel() + M.numel())
    gbs = out_bytes / (ms / 1e3) / 1e9
    return {"envs": n_envs, "ms": ms, "output_bytes": out_bytes, "output_GB_per_s": gbs,
            "frac_of_hbm_peak": gbs / PEAK_HBM_GBS,
            "finite": bool(torch.isfinite(J).all() and torch.isfinite(M).all())}


def run_hetero(params, n_envs, steps, fp64, preroll_steps):
    """Heterogeneous batch: ant-like, humanoid-like and arm+gripper+box environments in equal thirds,
    interleaved.  From the state an untimed pre-roll reaches, the same `steps` steps are timed with per-type
    launches, with the persistent launch, and with the mapping the autotuner picks on that state."""
    import torch
    from paper_2108_10470_amd import ags, workloads as W
    specs = [W.env_ant(), W.env_humanoid(), W.env_arm_box()]
    models = [ags.Model(s) for s in specs]
    env_model = [e % 3 for e in range(n_envs)]
    counts = [env_model.count(k) for k in range(3)]
    n_act = preroll_steps + steps
    init = [W.initial_state(specs[k], counts[k], 0) for k in range(3)]
    acts = [W.actuation(specs[k], counts[k], n_act, 0).astype(np.float32) for k in range(3)]
    roots, dofs, act_cols = [], [], []
    seen = [0, 0, 0]
    for e in range(n_envs):
        k = env_model[e]
        i = seen[k]
        seen[k] += 1
        roots.append(init[k][0][i].reshape(-1, 13))
        dofs.append(init[k][1][i].reshape(-1, 2))
        act_cols.append(acts[k][:, i])
    dev = "cuda:0"
    r0 = torch.tensor(np.concatenate(roots), dtype=torch.float32, device=dev)
    d0 = torch.tensor(np.concatenate(dofs), dtype=torch.float32, device=dev)
    a = torch.tensor(np.concatenate(act_cols, axis=1), dtype=torch.float32, device=dev)
    out = {"workload": f"{n_envs} envs: ant-like, humanoid-like and arm+gripper+box (capsule-box and box-plane "
                       f"contacts) in equal thirds, interleaved; {steps} steps timed after an untimed "
                       f"{preroll_steps}-step pre-roll", "envs": n_envs, "steps": steps,
           "dtype": "f64" if fp64 else "f32"}
    stream = torch.cuda.current_stream()
    pre = ags.Sim(models, env_model, params, device=dev, fp64=fp64)
    pre.root_state.copy_(r0)
    pre.dof_state.copy_(d0)
    for t in range(preroll_steps):
        pre.bind(ags.DOF_ACTUATION, a[t])
        pre.step()
    torch.cuda.synchronize()
    rp, dp = pre.root_state.clone(), pre.dof_state.clone()
    del pre

    def timed(**mapping):
        sim = ags.Sim(models, env_model, params, device=dev, fp64=fp64, **mapping)
        for rep in range(2):  # the first pass warms up
            sim.root_state.copy_(rp)
            sim.dof_state.copy_(dp)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for t in range(steps):
                sim.bind(ags.DOF_ACTUATION, a[preroll_steps + t])
                sim.step()
            e1.record(stream)
            torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        return {"ms_per_step": ms, "env_steps_per_s": n_envs / (ms / 1e3),
                "finite": bool(torch.isfinite(sim.root_state).all())}

    out["per_type"] = timed(persistent=False)
    out["persistent"] = timed(persistent=True)
    lanes, per, ms = ags.autotune(models, env_model, params, rp, dp, a[preroll_steps].contiguous(), fp64=fp64,
                                  n_steps=10)
    out["autotuned"] = {"lanes_per_env": lanes, "persistent": per, "autotuner_ms_per_step": ms,
                        **timed(persistent=per, lanes_per_env=lanes)}
    return out


def run_hand(n_envs, steps, fp64):
    """Scale workload: hand-like 24-DOF tree holding a free cube, PD drive toward targets re-drawn every
    step, capsule-box and box-plane contacts, 12 Gauss-Seidel sweeps; forward steps only."""
    import torch
    from paper_2108_10470_amd import ags, workloads as W
    env = W.env_hand_cube()
    p = W.HAND_PARAMS
    sim = ags.Sim([ags.Model(env)], [0] * n_envs, p, device="cuda:0", fp64=fp64, pd=True)
    root, dof = W.initial_state(env, n_envs, 0)
    r0 = torch.tensor(root.reshape(-1, 13), dtype=torch.float32, device="cuda:0")
    d0 = torch.tensor(dof.reshape(-1, 2), dtype=torch.float32, device="cuda:0")
    tg = torch.tensor(W.pd_targets(env, n_envs, steps, 0).reshape(steps, -1), dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    sim.root_state.copy_(r0)
    sim.dof_state.copy_(d0)
    for t in range(min(5, steps)):
        sim.bind(ags.DOF_POS_TARGET, tg[t])
        sim.step()
    sim.root_state.copy_(r0)
    sim.dof_state.copy_(d0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for t in range(steps):
        sim.bind(ags.DOF_POS_TARGET, tg[t])
        sim.step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return {"workload": f"hand-like 24-DOF tree + free cube, {n_envs} envs, PD targets re-drawn each step, "
                        "capsule-box and box-plane contacts, 12 sweeps", "envs": n_envs, "steps": steps,
            "dtype": "f64" if fp64 else "f32", "ms_per_step": ms, "env_steps_per_s": n_envs / (ms / 1e3),
            "finite": bool(torch.isfinite(sim.root_state).all() and torch.isfinite(sim.dof_state).all())}


def run_hand_fwd_bwd(n_envs, steps, fp64, every):
    """Hand + cube fwd+bwd: rollout driven by PD position targets (re-drawn each step), FP32 adjoint,
    loss = sum over envs of the final cube x position, gradient w.r.t. every target."""
    import torch
    from paper_2108_10470_amd import ags, workloads as W
    env = W.env_hand_cube()
    root, dof = W.initial_state(env, n_envs, 0)
    r0 = torch.tensor(root.reshape(-1, 13), dtype=torch.float32, device="cuda:0")
    d0 = torch.tensor(dof.reshape(-1, 2), dtype=torch.float32, device="cuda:0")
    tg = torch.tensor(W.pd_targets(env, n_envs, steps, 0).reshape(steps, -1), dtype=torch.float32, device="cuda:0")
    out = run_fwd_bwd(env, W.HAND_PARAMS, n_envs, fp64, tg, r0, d0, every, reps=1, adjoint_precision=32,
                      control=ags.DOF_POS_TARGET)
    out["loss"] = "sum over envs of the final cube x position (gradient w.r.t. PD targets)"
    return out


def cpu_baseline(env, params, root, dof, acts, n_envs, n_steps, n_envs_1, n_steps_1):
    """The FP64 oracle on the host over a bounded sample of the timed window: the GPU's state at the window's
    start (envs [0, n_envs)) stepped n_steps times with the window's actions, on every thread of the host's
    CPU share, and a smaller sample on one thread."""
    from oracle import oracle as O
    oe = O.OracleEnv(env)
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    threads = max(1, min(16, avail))  # the GPU machine's CPU share is 16 cores, whatever the machine shows

    def timed(n, k, nt):
        r, d = root[:n].copy(), dof[:n].copy()
        t0 = time.perf_counter()
        for t in range(k):
            o = oe.step(params, r, d, acts[t][:n], n_threads=nt)
            r, d = o["root"], o["dof"]
        return n * k / (time.perf_counter() - t0), time.perf_counter() - t0

    v, dt = timed(n_envs, n_steps, threads)
    v1, dt1 = timed(n_envs_1, n_steps_1, 1)
    return {"value": v, "unit": "env-steps/s", "cores": threads, "kind": "oracle",
            "value_1core": v1, "host_cpus_visible": avail,
            "sample": f"the GPU's FP32 state at the timed window's start, {n_envs} humanoid envs x {n_steps} env-steps "
                      f"with the window's actions on {threads} threads ({dt:.1f} s); one thread: {n_envs_1} envs x "
                      f"{n_steps_1} steps ({dt1:.1f} s); FP64"}


def run_ant_grad(fp64, reps):
    """Differentiation workload: 4096 ant-like envs from the seeded start, 64-step rollout with a checkpoint
    every 16 steps, loss = sum over envs of the final torso x position, gradient w.r.t. all 64 x 8 actions
    per env (FP32 adjoint)."""
    import torch
    from paper_2108_10470_amd import workloads as W
    env = W.env_ant()
    params = W.SimParams()
    E, T, every = 4096, 64, 16
    root, dof = W.initial_state(env, E, 0)
    r0 = torch.tensor(root.reshape(-1, 13), dtype=torch.float32, device="cuda:0")
    d0 = torch.tensor(dof.reshape(-1, 2), dtype=torch.float32, device="cuda:0")
    acts = torch.tensor(W.actuation(env, E, T, 0).astype(np.float32).reshape(T, -1), device="cuda:0")
    out = run_fwd_bwd(env, params, E, fp64, acts, r0, d0, every, reps, adjoint_precision=32)
    out["workload"] = "ant-like, 4096 envs, 64-step rollout from the seeded start, checkpoints every 16"
    return out


def phase_report(env, params, E, P, actions_dev, root_stand, dof_stand, steps=5):
    """Per-phase shader-clock cycles per substep (mean over envs) of the step kernel (FP64 and FP32) and of the
    adjoint's recomputation in its dense form (composite inertias + M~ + Cholesky; J rows + W = M~^-1 J^T by
    triangular solves; A = J W^T on the matrix cores), FP64 and FP32 adjoint, on the pre-rolled window."""
    import torch
    from paper_2108_10470_amd import ags
    root0, dof0 = preroll(env, params, E, P, actions_dev, root_stand, dof_stand)
    out = {"envs": E, "preroll_steps": P}
    names = ["controls", "forward", "inward", "outward", "vstar", "narrow", "rows", "responses", "pgs", "outputs"]
    for fp64 in (True, False):
        sim = ags.Sim([ags.Model(env)], [0] * E, params, device="cuda:0", fp64=fp64, phase_cycles=True)
        sim.root_state.copy_(root0)
        sim.dof_state.copy_(dof0)
        acc = torch.zeros(E, len(names), dtype=torch.float64, device="cuda:0")
        for t in range(steps):
            sim.bind(ags.DOF_ACTUATION, actions_dev[P + t])
            sim.step()
            acc += sim.dbg_cycles.double()
        torch.cuda.synchronize()
        c = (acc / steps).mean(0).cpu().numpy() / params.substeps
        out[f"step_{'fp64' if fp64 else 'fp32'}_cycles_per_substep"] = {n: round(float(v)) for n, v in zip(names, c)}
    an = ["recompute_other", "recompute_gauss_seidel", "reverse_gauss_seidel", "reverse_dense_products",
          "reverse_mass_terms", "reverse_rnea", "reverse_rows", "reverse_integration", "dense_crba_cholesky",
          "dense_rows_J_W", "dense_delassus_mfma"]
    for prec in (64, 32):
        sim = ags.Sim([ags.Model(env)], [0] * E, params, device="cuda:0", fp64=True, adjoint_precision=prec)
        cyc = torch.zeros((E, len(an)), dtype=torch.int64, device="cuda:0")
        sim.bind(ags.DEBUG_ADJ_CYCLES, cyc)
        acc = torch.zeros(E, len(an), dtype=torch.float64, device="cuda:0")
        aa = torch.zeros(actions_dev[0].shape, dtype=torch.float32, device="cuda:0")
        for t in range(3):
            ra = torch.zeros_like(root0)
            ra[:, 0] = 1.0
            sim.step_backward(root0, dof0, actions_dev[P + t], ra, torch.zeros_like(dof0), aa)
            acc += cyc.double()
        torch.cuda.synchronize()
        # one call recomputes 2 S - 1 substeps (S - 1 to reach the last, then each again before its reverse)
        c = (acc / 3).mean(0).cpu().numpy() / (2 * params.substeps - 1)
        out[f"adjoint_fp{prec}_cycles_per_recomputed_substep"] = {
            n: round(float(v)) for n, v in zip(an, c) if n.startswith("recompute") or n.startswith("dense")}
    print(json.dumps(out), flush=True)


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
    E, K, Wm, P = args.envs, args.steps, args.warmup, args.preroll
    root, dof = W.initial_state(env, E, 0)
    n_act = P + max(Wm + K, args.fwd_bwd_steps, args.rows_ref_steps - P)
    acts = W.actuation(env, E, n_act, 0).astype(np.float32)
    actions_dev = torch.from_numpy(acts).to("cuda:0").reshape(n_act, -1)
    actions_dev = [actions_dev[t] for t in range(n_act)]
    root_stand = torch.from_numpy(root.reshape(-1, 13).astype(np.float32)).to("cuda:0")
    dof_stand = torch.from_numpy(dof.reshape(-1, 2).astype(np.float32)).to("cuda:0")
    print(f"[bench] humanoid envs={E} preroll={P} warmup={Wm} steps={K}", file=sys.stderr, flush=True)
    if args.calib_copy_mb:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.phase_report:
        phase_report(env, params, E, P, actions_dev, root_stand, dof_stand)
        return
    root0, dof0 = preroll(env, params, E, P, actions_dev, root_stand, dof_stand)
    win_actions = actions_dev[P:]

    variants = {"both": [True, False], "fp64": [True], "fp32": [False]}[args.precision]
    res = {}
    for fp64 in variants:
        name = "fp64" if fp64 else "fp32"
        r = run_gpu(env, params, E, K, Wm, fp64, win_actions, root0, dof0)
        r["rows"] = None if args.no_rows else mean_rows(env, params, E, Wm + K, fp64, win_actions, root0, dof0,
                                                         skip=Wm)
        res[name] = r
        print(f"[bench] {name}: {K} steps in {r['total_ms']:.1f} ms, launch mean {r['launch_ms'].mean():.3f} ms, "
              f"rows/substep {r['rows']}, graph {r['graph_ms']} vs eager {r['eager_same_steps_ms']} ms/step, "
              f"finite {r['finite']}", file=sys.stderr, flush=True)
    rows_ref = None
    if not args.no_rows and args.rows_ref_steps > 0:
        rows_ref = mean_rows(env, params, E, args.rows_ref_steps, False, actions_dev, root_stand, dof_stand)
        print(f"[bench] rows/substep over steps 0-{args.rows_ref_steps} from the standing start: {rows_ref}",
              file=sys.stderr, flush=True)

    head = "fp64" if "fp64" in res else "fp32"
    hetero = None
    if not args.no_hetero:
        hetero = run_hetero(params, args.hetero_envs, args.hetero_steps, head == "fp64", args.hetero_preroll)
        print(f"[bench] heterogeneous batch: {json.dumps(hetero)}", file=sys.stderr, flush=True)
    hand = None
    if not args.no_hand:
        hand = run_hand(args.hand_envs, args.hand_steps, head == "fp64")
        print(f"[bench] hand: {json.dumps(hand)}", file=sys.stderr, flush=True)
        if not args.no_fwd_bwd:
            hand["fwd_bwd"] = run_hand_fwd_bwd(args.hand_envs, args.hand_steps, head == "fp64", args.fwd_bwd_every)
            print(f"[bench] hand fwd+bwd: {json.dumps(hand['fwd_bwd'])}", file=sys.stderr, flush=True)
    tgs = None
    if not args.no_tgs:  # the temporal Gauss-Seidel variant of the solver, same workload and precision
        import dataclasses
        r = run_gpu(env, dataclasses.replace(params, solver=1), E, K, Wm, head == "fp64", win_actions, root0, dof0)
        tgs = {"env_steps_per_s": E * K / (r["total_ms"] / 1e3), "ms_per_step": r["total_ms"] / K,
               "launch_ms": float(r["launch_ms"].mean()), "finite": r["finite"], "dtype": head.replace("fp", "f")}
        print(f"[bench] tgs: {json.dumps(tgs)}", file=sys.stderr, flush=True)
    randomized = None
    if not args.no_tgs:  # every property tensor bound (masses, gains, limits, friction, gravity per env)
        r = run_gpu(env, params, E, K, Wm, head == "fp64", win_actions, root0, dof0,
                    props=W.random_properties(env, params, E, seed=0))
        randomized = {"env_steps_per_s": E * K / (r["total_ms"] / 1e3), "ms_per_step": r["total_ms"] / K,
                      "launch_ms": float(r["launch_ms"].mean()), "finite": r["finite"],
                      "finite_env_fraction": r["finite_frac"], "dtype": head.replace("fp", "f"),
                      "note": "with the paper's damping draw (x loguniform[0.3, 3]) a few humanoids diverge within "
                              "~800 steps; the FP64 oracle stepped from the same state diverges the same way"}
        print(f"[bench] randomized properties: {json.dumps(randomized)}", file=sys.stderr, flush=True)
    jacmass = run_jacmass(env, params, E, root0, dof0)
    print(f"[bench] jacobian+mass: {json.dumps(jacmass)}", file=sys.stderr, flush=True)
    fwd_bwd = None
    if not args.no_fwd_bwd:
        T = args.fwd_bwd_steps
        acts_fb = torch.stack(win_actions[:T]).contiguous()
        fwd_bwd = run_fwd_bwd(env, params, E, head == "fp64", acts_fb, root0, dof0, args.fwd_bwd_every,
                              args.fwd_bwd_reps, adjoint_precision=32)
        print(f"[bench] fwd+bwd ({head} forward, f32 adjoint): {json.dumps(fwd_bwd)}", file=sys.stderr, flush=True)
        fb64 = run_fwd_bwd(env, params, E, head == "fp64", acts_fb, root0, dof0, args.fwd_bwd_every,
                           args.fwd_bwd_reps, adjoint_precision=64)
        print(f"[bench] fwd+bwd ({head} forward, f64 adjoint): {json.dumps(fb64)}", file=sys.stderr, flush=True)
        fwd_bwd["f64_adjoint"] = {k: fb64[k] for k in ("value", "ms_forward", "ms_backward", "adjoint_launch_ms")}
        if args.fwd_bwd_ckpt_every != args.fwd_bwd_every:
            fbc = run_fwd_bwd(env, params, E, head == "fp64", acts_fb, root0, dof0, args.fwd_bwd_ckpt_every,
                              args.fwd_bwd_reps, adjoint_precision=32)
            print(f"[bench] fwd+bwd ({head} forward, f32 adjoint, checkpoints every {args.fwd_bwd_ckpt_every}): "
                  f"{json.dumps(fbc)}", file=sys.stderr, flush=True)
            fwd_bwd["checkpointed"] = {k: fbc[k] for k in ("value", "checkpoint_every", "ms_forward", "ms_backward")}
        fwd_bwd["start"] = f"the state of the pre-roll ({P} steps from standing)"
        if not args.no_ant_grad:
            fwd_bwd["ant_differentiation"] = run_ant_grad(head == "fp64", args.fwd_bwd_reps)
            print(f"[bench] ant differentiation: {json.dumps(fwd_bwd['ant_differentiation'])}", file=sys.stderr,
                  flush=True)
    h = res[head]
    value = E * K / (h["total_ms"] / 1e3)
    t_launch = float(h["launch_ms"].mean()) / 1e3
    rows = h["rows"]  # None with --no-rows: the flop count needs the measured row count
    ach_tf = None if rows is None else E * (FLOPS_BASE + FLOPS_PER_ROW * rows) / t_launch / 1e12
    ach_gbs = E * BYTES_PER_ENV_STEP / t_launch / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "env-steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": h["total_ms"] / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": "humanoid-like, 4096 envs (13 capsules, free root + 21 revolute DOFs), "
                               "dt 1/60 s x 2 substeps, 8 PGS sweeps, actions U[-1,1] x 67.5; window after an "
                               f"untimed {P}-step pre-roll from the standing start (humanoids on the ground)",
                   "envs": E, "substeps": params.substeps, "pgs_iters": params.pgs_iters, "preroll_steps": P,
                   "tensors": "f32", "compute": head, "mean_rows_per_substep": rows,
                   "mean_rows_per_substep_steps_0_to_%d" % args.rows_ref_steps: rows_ref},
        "roofline": {"bound": "alu", "achieved": ach_tf, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": None if ach_tf is None else ach_tf / PEAK_VALU_TFLOPS, "traffic": measured_traffic(head),
                     "kernel": "step_kernel<double>" if head == "fp64" else "step_kernel<float>",
                     "launch_ms": t_launch * 1e3,
                     "hbm": {"achieved": ach_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach_gbs / PEAK_HBM_GBS,
                             "bytes_per_env_step": BYTES_PER_ENV_STEP},
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"},
        "fwd_bwd": fwd_bwd,
        "batching": hetero,
        "hand": hand,
        "jacobian_mass": jacmass,
        "tgs": tgs,
        "randomized_properties": randomized,
        "variants": {k: {"env_steps_per_s": E * K / (v["total_ms"] / 1e3), "ms_per_step": v["total_ms"] / K,
                         "launch_ms": float(v["launch_ms"].mean()), "mean_rows_per_substep": v["rows"],
                         "graph_ms_per_step": v["graph_ms"], "eager_ms_per_step_same_steps": v["eager_same_steps_ms"],
                         "graph_steps": v["graph_chunk"], "finite": v["finite"]} for k, v in res.items()},
    }
    if not args.no_cpu_baseline:
        wr = h["window_root"].double().cpu().numpy().reshape(E, env.n_actors, 13)
        wd = h["window_dof"].double().cpu().numpy().reshape(E, env.n_dof, 2)
        wa = acts[P + Wm:P + Wm + args.cpu_steps].astype(np.float64)
        out["cpu_baseline"] = cpu_baseline(W.as_f32(env), W.params_f32(params), wr, wd, wa,
                                           min(args.cpu_envs, E), min(args.cpu_steps, len(wa)),
                                           min(args.cpu_envs_1core, E), min(args.cpu_steps_1core, len(wa)))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
