"""Adjoint checks: gradients from the HIP adjoint against central finite differences of the FP64 oracle.

A loss L = sum(wr * root_after) + sum(wd * dof_after) with seeded weights is differentiated with
respect to the actuation, the DOF state and the free-root state of one env-step.  The oracle is fed
the same FP32-rounded inputs and perturbed by +-H in FP64.  An entry whose two perturbed steps do not
both take the discrete decisions of the unperturbed step (the oracle's mode hash: row set, bias
branches, every clamp) straddles a mode switch, where the step has no derivative; it is excluded
and counted.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O
from paper_2108_10470_amd import ags, workloads as W

H = 1e-6
RTOL = 1e-3


def entries(env):
    """(array, index) of every differentiated input of one env: actuation, DOF (q, qd), free-root
    (position, quaternion, linear and angular velocity)."""
    out = [("act", (j,)) for j in range(env.n_dof)]
    out += [("dof", (j, c)) for j in range(env.n_dof) for c in range(2)]
    for a, act in enumerate(env.actors):
        if act.links[0].joint == "free":
            out += [("root", (a, c)) for c in range(13)]
    return out


def fd_grads(oe, params, root, dof, act, wr, wd, n_threads=None):
    """Central differences of the loss for every entry of every env; NaN where the mode changes."""
    E = root.shape[0]
    ent = entries(oe.spec)
    n = len(ent)
    R = np.repeat(root[:, None], 2 * n + 1, axis=1).copy()
    D = np.repeat(dof[:, None], 2 * n + 1, axis=1).copy()
    A = np.repeat(act[:, None], 2 * n + 1, axis=1).copy()
    for k, (arr, idx) in enumerate(ent):
        for sgn, slot in ((1.0, 2 * k), (-1.0, 2 * k + 1)):
            tgt = {"act": A, "dof": D, "root": R}[arr]
            tgt[(slice(None), slot) + idx] += sgn * H
    o = oe.step(params, R.reshape(E * (2 * n + 1), *root.shape[1:]), D.reshape(E * (2 * n + 1), *dof.shape[1:]),
                A.reshape(E * (2 * n + 1), -1), n_threads=n_threads)
    L = ((o["root"].reshape(E, 2 * n + 1, -1) * wr.reshape(E, 1, -1)).sum(-1)
         + (o["dof"].reshape(E, 2 * n + 1, -1) * wd.reshape(E, 1, -1)).sum(-1))
    mode = o["mode"].reshape(E, 2 * n + 1)
    g = (L[:, 0:2 * n:2] - L[:, 1:2 * n:2]) / (2 * H)
    same = (mode[:, 0:2 * n:2] == mode[:, 2 * n:]) & (mode[:, 1:2 * n:2] == mode[:, 2 * n:])
    return np.where(same, g, np.nan), ent


def gpu_grads(env, params, root, dof, act, wr, wd, fp64, device="cuda:0"):
    """HIP adjoint of the same loss; returns (grad per entry, status per env)."""
    E = root.shape[0]
    model = ags.Model(env)
    sim = ags.Sim([model], [0] * E, params, device=device, fp64=fp64)
    f32 = dict(dtype=torch.float32, device=device)
    rs = torch.tensor(root.reshape(-1, 13), **f32)
    ds = torch.tensor(dof.reshape(-1, 2), **f32)
    ac = torch.tensor(act.reshape(-1), **f32)
    ra = torch.tensor(wr.reshape(-1, 13), **f32)
    da = torch.tensor(wd.reshape(-1, 2), **f32)
    aa = torch.zeros(env.n_dof * E, **f32)
    st = torch.full((E,), -1, dtype=torch.int32, device=device)
    sim.step_backward(rs, ds, ac, ra, da, aa, st)
    torch.cuda.synchronize()
    ra = ra.double().cpu().numpy().reshape(root.shape)
    da = da.double().cpu().numpy().reshape(dof.shape)
    aa = aa.double().cpu().numpy().reshape(act.shape)
    out = np.zeros((E, len(entries(env))))
    for k, (arr, idx) in enumerate(entries(env)):
        src = {"act": aa, "dof": da, "root": ra}[arr]
        out[:, k] = src[(slice(None),) + idx]
    return out, st.cpu().numpy()


def compare(g, fd, floor_frac):
    """Per-env worst ratio |g - fd| / (RTOL |fd| + floor_frac max|fd|) over the entries away from switches."""
    ok = ~np.isnan(fd)
    scale = np.nanmax(np.abs(fd), axis=1, keepdims=True)
    ratio = np.abs(g - fd) / (RTOL * np.abs(fd) + floor_frac * scale + 1e-30)
    ratio = np.where(ok, ratio, 0.0)
    return ratio.max(axis=1), ok


def normwise(g, fd):
    """Per-env relative error of the gradient vector, |g - fd| / |fd|, over the entries away from switches
    (no floor: the reading of a relative gradient error that does not depend on an absolute scale)."""
    ok = ~np.isnan(fd)
    d = np.where(ok, g - fd, 0.0)
    f = np.where(ok, fd, 0.0)
    return np.linalg.norm(d, axis=1) / (np.linalg.norm(f, axis=1) + 1e-300)


def f32_inputs(env, params, n_envs, steps_before, seed=0):
    """Seeded start states rolled out by the oracle for `steps_before` steps, rounded to FP32, with the
    next step's actions and seeded loss weights."""
    env = W.as_f32(env)
    params = W.params_f32(params)
    oe = O.OracleEnv(env)
    root, dof = W.initial_state(env, n_envs, seed)
    acts = W.actuation(env, n_envs, steps_before + 1, seed)
    for t in range(steps_before):
        o = oe.step(params, root, dof, acts[t])
        root, dof = o["root"], o["dof"]
    r32 = lambda x: x.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(seed + 17)
    wr = r32(rng.standard_normal(root.shape))
    wd = r32(rng.standard_normal(dof.shape))
    return env, params, oe, r32(root), r32(dof), r32(acts[steps_before]), wr, wd


def fd_rollout(oe, params, root0, dof0, acts, n_threads=None, h=None, targets=False, actor=0, weights=None):
    """Central differences (step h, default H) of L = sum over envs of actor `actor`'s final root x
    position after the rollout of acts (T, E, D) (the actuation, or with targets=True the PD position
    targets with zero actuation), with respect to every entry; NaN where any step's mode changes.
    Also returns the mode of every step of the unperturbed rollout (E, T)."""
    H_ = H if h is None else h
    T, E, nd = acts.shape
    n = T * nd
    C = 2 * n + 1
    R = np.repeat(root0[:, None], C, axis=1).reshape(E * C, *root0.shape[1:])
    D = np.repeat(dof0[:, None], C, axis=1).reshape(E * C, *dof0.shape[1:])
    A = np.repeat(acts[:, :, None], C, axis=2).copy()  # T, E, C, nd
    for t in range(T):
        for j in range(nd):
            k = t * nd + j
            A[t, :, 2 * k, j] += H_
            A[t, :, 2 * k + 1, j] -= H_
    mode = np.zeros(E * C, dtype=np.uint64)
    base_modes = np.zeros((E, T), dtype=np.uint64)
    with np.errstate(over="ignore"):
        for t in range(T):
            ctl = A[t].reshape(E * C, nd)
            if targets:
                o = oe.step(params, R, D, np.zeros_like(ctl), pos_tgt=ctl, n_threads=n_threads)
            else:
                o = oe.step(params, R, D, ctl, n_threads=n_threads)
            R, D = o["root"], o["dof"]
            mode = (mode * np.uint64(1099511628211)) ^ o["mode"]
            base_modes[:, t] = o["mode"].reshape(E, C)[:, 2 * n]
    if weights is None:
        L = R.reshape(E, C, -1, 13)[:, :, actor, 0]
    else:  # L = sum(wr * final root states) + sum(wd * final DOF states)
        wr, wd = weights
        L = ((R.reshape(E, C, -1) * wr.reshape(E, 1, -1)).sum(-1) + (D.reshape(E, C, -1) * wd.reshape(E, 1, -1)).sum(-1))
    mode = mode.reshape(E, C)
    g = (L[:, 0:2 * n:2] - L[:, 1:2 * n:2]) / (2 * H_)
    same = (mode[:, 0:2 * n:2] == mode[:, 2 * n:]) & (mode[:, 1:2 * n:2] == mode[:, 2 * n:])
    return np.where(same, g, np.nan).reshape(E, T, nd), base_modes


def gpu_trajectory(env, params, root0, dof0, acts, fp64, device="cuda:0", targets=False):
    """States of the GPU rollout of acts (T, E, D) before every step and after the last:
    roots (T + 1, E, A, 13), dofs (T + 1, E, D, 2)."""
    T, E, nd = acts.shape
    sim = ags.Sim([ags.Model(env)], [0] * E, params, device=device, fp64=fp64, pd=targets)
    f32 = dict(dtype=torch.float32, device=device)
    sim.root_state.copy_(torch.tensor(root0.reshape(-1, 13), **f32))
    sim.dof_state.copy_(torch.tensor(dof0.reshape(-1, 2), **f32))
    ctl = sim.pos_target if targets else sim.actuation
    roots, dofs = [], []
    for t in range(T):
        roots.append(sim.root_state.double().cpu().numpy().reshape(root0.shape))
        dofs.append(sim.dof_state.double().cpu().numpy().reshape(dof0.shape))
        ctl.copy_(torch.tensor(acts[t].reshape(-1), **f32))
        sim.step()
    torch.cuda.synchronize()
    roots.append(sim.root_state.double().cpu().numpy().reshape(root0.shape))
    dofs.append(sim.dof_state.double().cpu().numpy().reshape(dof0.shape))
    return np.stack(roots), np.stack(dofs)


def gpu_rollout_grad(env, params, root0, dof0, acts, every, fp64, device="cuda:0", targets=False, actor=0,
                     adjoint_precision=0, weights=None):
    """The same gradient through ags.rollout (checkpoints every `every` steps) and torch autograd."""
    T, E, nd = acts.shape
    sim = ags.Sim([ags.Model(env)], [0] * E, params, device=device, fp64=fp64, pd=targets,
                  adjoint_precision=adjoint_precision)
    f32 = dict(dtype=torch.float32, device=device)
    a = torch.tensor(acts.reshape(T, E * nd), **f32).requires_grad_(True)
    r0 = torch.tensor(root0.reshape(-1, 13), **f32)
    d0 = torch.tensor(dof0.reshape(-1, 2), **f32)
    root, dof = ags.rollout(sim, a, r0, d0, every=every,
                            control=ags.DOF_POS_TARGET if targets else ags.DOF_ACTUATION)
    if weights is None:
        loss = root.view(E, env.n_actors, 13)[:, actor, 0].sum()
    else:
        wr, wd = (torch.tensor(w.reshape(-1), **f32) for w in weights)
        loss = (root.reshape(-1) * wr).sum() + (dof.reshape(-1) * wd).sum()
    loss.backward()
    torch.cuda.synchronize()
    return a.grad.double().cpu().numpy().reshape(T, E, nd).transpose(1, 0, 2), root.detach().double().cpu().numpy()
