"""HIP path vs FP64 oracle, one env-step from identical FP32 states (see tests/parity.py)."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2108_10470_amd import ags, workloads as W

from . import parity as PT

pytestmark = pytest.mark.gpu

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")


def _report(name, summary):
    print(name, json.dumps(summary), flush=True)
    if os.path.isdir(OUT):
        with open(os.path.join(OUT, "parity.jsonl"), "a") as f:
            f.write(json.dumps({"case": name, **summary}) + "\n")


def _assert_pass(s):
    assert s["rows_mismatch_not_near"] == 0, s
    for k in ("qdd_free", "q", "lambda"):
        assert s[k + "_pass_rate"] == 1.0, (k, s)


def _assert_fp32(s):
    """FP32 compute: FP32 rounding amplified by the conditioning of M~ and of the Delassus matrix moves
    accelerations and impulses by more than 1e-4 relative (measured up to ~2e-2 on the ant's friction
    impulses), so the FP32 variant is held to identical row sets away from switches and positions within
    ten times the FP64 bound; the other ratios are reported."""
    assert s["rows_mismatch_not_near"] == 0, s
    assert s["q_max_ratio"] <= 10.0, s


def test_pendulum_free_swing():
    env = W.EnvSpec("pend", [W.pendulum()], [])
    p = W.SimParams()
    E = 16
    root, dof = W.initial_state(env, E)
    dof[:, 0, 0] = np.linspace(-2.5, 2.5, E)
    dof[:, 0, 1] = np.linspace(3.0, -3.0, E)
    g, o = PT.run(env, p, root, dof, np.zeros((E, 1)))
    s = PT.summarize(PT.compare(env, p, g, o))
    _report("pendulum", s)
    _assert_pass(s)
    # closed form of the oracle pin: qdd = -m g l_c sin q / I_pivot is what both sides must reproduce
    assert np.all(g["row_count"] == 0)


@pytest.mark.parametrize("lanes", [32, 64])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_humanoid_parity_from_oracle_states(fp64, lanes):
    env = W.env_humanoid()
    p = W.SimParams()
    oe, root, dof, act = PT.oracle_states(env, p, n_envs=32, n_steps=120, every=8)
    g, o = PT.run(env, p, root, dof, act, oe=oe, fp64=fp64, lanes_per_env=lanes)
    c = PT.compare(env, p, g, o)
    s = PT.summarize(c)
    s["mean_rows"] = float(o["row_count"].mean())
    s["max_rows"] = int(o["row_count"].max())
    _report(f"humanoid_{'fp64' if fp64 else 'fp32'}_l{lanes}", s)
    _assert_pass(s) if fp64 else _assert_fp32(s)


@pytest.mark.parametrize("lanes", [32, 64])
@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_ant_parity_every_step(fp64, lanes):
    """Ant-like quadruped, 64 envs, every one of 100 steps (states from the oracle rollout)."""
    env = W.env_ant()
    p = W.SimParams()
    oe, root, dof, act = PT.oracle_states(env, p, n_envs=64, n_steps=100, every=1)
    g, o = PT.run(env, p, root, dof, act, oe=oe, fp64=fp64, lanes_per_env=lanes)
    c = PT.compare(env, p, g, o)
    s = PT.summarize(c)
    s["mean_rows"] = float(o["row_count"].mean())
    _report(f"ant_{'fp64' if fp64 else 'fp32'}_l{lanes}", s)
    _assert_pass(s) if fp64 else _assert_fp32(s)


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_hand_cube_parity(fp64):
    """Hand-like tree (24 PD-driven DOFs) holding a free cube: capsule-box contacts with the palm and
    fingers, 12 Gauss-Seidel sweeps, seeded PD targets; states from a 60-step oracle rollout."""
    env = W.env_hand_cube()
    p = W.HAND_PARAMS
    E, T, every = 16, 60, 6
    envf, pf = W.as_f32(env), W.params_f32(p)
    oe = O.OracleEnv(envf)
    root, dof = W.initial_state(envf, E, 0)
    tg = W.pd_targets(envf, E, T, 0)
    act = np.zeros((E, env.n_dof))
    roots, dofs, tgts = [], [], []
    for t in range(T):
        if t % every == 0:
            roots.append(root)
            dofs.append(dof)
            tgts.append(tg[t])
        o = oe.step(pf, root, dof, act, pos_tgt=tg[t])
        root, dof = o["root"], o["dof"]
    root, dof, tg = np.concatenate(roots), np.concatenate(dofs), np.concatenate(tgts)
    g, o = PT.run(env, p, root, dof, np.zeros((root.shape[0], env.n_dof)), oe=oe, pos_tgt=tg, fp64=fp64)
    s = PT.summarize(PT.compare(env, p, g, o))
    s["mean_rows"] = float(o["row_count"].mean())
    s["max_rows"] = int(o["row_count"].max())
    _report(f"hand_cube_{'fp64' if fp64 else 'fp32'}", s)
    assert np.isfinite(g["root"]).all() and np.isfinite(g["dof"]).all()
    _assert_pass(s) if fp64 else _assert_fp32(s)
