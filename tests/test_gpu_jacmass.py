"""Jacobian and generalized mass-matrix tensors (Section 2.3, Table 1) on the GPU against the oracle: the
oracle's Jacobian is the rigid-body velocity map evaluated column by column and its mass matrix is CRBA,
both pinned on the CPU (FK differences, the kinetic-energy form)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2108_10470_amd import ags, workloads as W

pytestmark = pytest.mark.gpu

OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "gpurun_out")
ATOL, RTOL = 1e-5, 1e-4


def _report(name, d):
    print(name, json.dumps(d), flush=True)
    if os.path.isdir(OUT):
        with open(os.path.join(OUT, "parity.jsonl"), "a") as f:
            f.write(json.dumps({"case": name, **d}) + "\n")


def _poses(env, n, seed):
    """n envs at seeded poses: joints moved by U[-0.5, 0.5] from the initial pose, free roots turned to
    random orientations and moved by U[-1, 1] m; rounded to FP32 (the tensors' type)."""
    root, dof = W.initial_state(env, n, seed)
    rng = np.random.default_rng(seed + 1000)
    dof[:, :, 0] += rng.uniform(-0.5, 0.5, dof.shape[:2])
    for ai, a in enumerate(env.actors):
        if not a.fixed_base:
            q = rng.normal(size=(n, 4))
            root[:, ai, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
            root[:, ai, 0:3] += rng.uniform(-1.0, 1.0, (n, 3))
    r32 = lambda x: x.astype(np.float32).astype(np.float64)
    return r32(root), r32(dof)


def _gpu(sim, model, root, dof):
    f32 = dict(dtype=torch.float32, device="cuda:0")
    sim.root_state.copy_(torch.tensor(root.reshape(-1, 13), **f32))
    sim.dof_state.copy_(torch.tensor(dof.reshape(-1, 2), **f32))
    J, M = sim.jacobian_mass(model)
    torch.cuda.synchronize()
    return J.double().cpu().numpy(), M.double().cpu().numpy()


def _check(name, env, oe, root, dof, J, M, envs):
    worst_j = worst_m = 0.0
    for i, e in enumerate(envs):
        Jo = oe.jacobian(root[e], dof[e])
        Mo = oe.mass_matrix(root[e], dof[e])
        worst_j = max(worst_j, float((np.abs(J[i] - Jo) / (ATOL + RTOL * np.abs(Jo))).max()))
        worst_m = max(worst_m, float((np.abs(M[i] - Mo) / (ATOL + RTOL * np.abs(Mo))).max()))
    d = {"envs_checked": len(envs), "n_v": oe.n_v, "n_bodies": oe.n_bodies, "jacobian_worst_ratio": worst_j,
         "mass_worst_ratio": worst_m}
    _report(name, d)
    assert worst_j <= 1.0 and worst_m <= 1.0, d


@pytest.mark.parametrize("make", [W.env_humanoid, W.env_arm_box, W.env_hand_cube, W.env_ant],
                         ids=["humanoid", "arm_box", "hand_cube", "ant"])
def test_jacobian_and_mass_matrix_match_oracle(make):
    """Every entry of the Jacobian (n_links x 6 x n_v) and of M (n_v x n_v) of 24 envs at seeded poses,
    within 1e-5 + 1e-4 |oracle|; M symmetric with a positive spectrum."""
    env = W.as_f32(make())
    oe = O.OracleEnv(env)
    n = 24
    root, dof = _poses(env, n, 3)
    sim = ags.Sim([ags.Model(env)], [0] * n, W.SimParams(), device="cuda:0")
    J, M = _gpu(sim, 0, root, dof)
    assert J.shape == (n, oe.n_bodies, 6, oe.n_v) and M.shape == (n, oe.n_v, oe.n_v)
    assert np.isfinite(J).all() and np.isfinite(M).all()
    assert (M == M.transpose(0, 2, 1)).all()
    assert np.linalg.eigvalsh(M).min() > 0
    _check(f"jacmass_{make.__name__}", env, oe, root, dof, J, M, range(n))


def test_jacobian_mass_per_model_of_a_heterogeneous_sim():
    """Ant-like, humanoid-like and arm+box envs interleaved: each model's call returns its own envs, in
    env order, at their own states."""
    specs = [W.as_f32(W.env_ant()), W.as_f32(W.env_humanoid()), W.as_f32(W.env_arm_box())]
    n = 8
    env_model = [e % 3 for e in range(3 * n)]
    states = [_poses(s, n, 7 + k) for k, s in enumerate(specs)]
    roots, dofs = [], []
    for e in range(3 * n):
        k, i = e % 3, e // 3
        roots.append(states[k][0][i].reshape(-1, 13))
        dofs.append(states[k][1][i].reshape(-1, 2))
    sim = ags.Sim([ags.Model(s) for s in specs], env_model, W.SimParams(), device="cuda:0")
    f32 = dict(dtype=torch.float32, device="cuda:0")
    sim.root_state.copy_(torch.tensor(np.concatenate(roots), **f32))
    sim.dof_state.copy_(torch.tensor(np.concatenate(dofs), **f32))
    for k, s in enumerate(specs):
        J, M = sim.jacobian_mass(k)
        torch.cuda.synchronize()
        _check(f"jacmass_hetero_model{k}", s, O.OracleEnv(s), states[k][0], states[k][1],
               J.double().cpu().numpy(), M.double().cpu().numpy(), range(n))


def test_jacobian_mass_full_batch_sampled():
    """4096 humanoid-like envs (the step benchmark's batch size): every 128th env against the oracle, and
    for every 16th env the kinetic energy 1/2 qd^T M qd at a random qd equal to the one summed over the
    bodies from the Jacobian's velocities and the mass properties (a property that holds at any size)."""
    env = W.as_f32(W.env_humanoid())
    oe = O.OracleEnv(env)
    n = 4096
    root, dof = _poses(env, n, 11)
    sim = ags.Sim([ags.Model(env)], [0] * n, W.SimParams(), device="cuda:0")
    J, M = _gpu(sim, 0, root, dof)
    sample = list(range(0, n, 128))
    _check("jacmass_humanoid_4096_sampled", env, oe, root, dof, J[sample], M[sample], sample)
    # energy identity: links' COM velocity = origin velocity + w x (R c)
    m, com, Ic = oe.mass_props()
    R, _ = zip(*[oe.fk(root[e], dof[e]) for e in range(0, n, 16)])
    rng = np.random.default_rng(2)
    qd = rng.normal(size=(n, oe.n_v))
    T_M = 0.5 * np.einsum("ei,eij,ej->e", qd, M, qd)
    V = np.einsum("ebrk,ek->ebr", J, qd)
    for j, e in enumerate(range(0, n, 16)):
        v, w = V[e, :, :3], V[e, :, 3:]
        rc = np.einsum("bij,bj->bi", R[j], com)
        vc = v + np.cross(w, rc)
        Iw = np.einsum("bij,bjk,blk->bil", R[j], Ic, R[j])
        T_J = 0.5 * (m * (vc * vc).sum(1)).sum() + 0.5 * np.einsum("bi,bij,bj->", w, Iw, w)
        assert abs(T_J - T_M[e]) <= 1e-4 * abs(T_J) + 1e-5, (e, T_J, T_M[e])
    assert np.isfinite(M).all() and (np.linalg.eigvalsh(M[::64]).min() > 0)


def test_single_output_calls_equal_the_combined_call():
    """Asking for J alone or M alone (the kernel then skips the other output's phases) returns bitwise
    what the call asking for both returns; asking for neither output, or for a model the sim does not
    have, is an error."""
    env = W.as_f32(W.env_hand_cube())
    n = 33
    root, dof = _poses(env, n, 5)
    sim = ags.Sim([ags.Model(env)], [0] * n, W.SimParams(), device="cuda:0")
    J, M = _gpu(sim, 0, root, dof)
    J1, M1 = sim.jacobian_mass(0, jacobian=True, mass=False)
    J2, M2 = sim.jacobian_mass(0, jacobian=False, mass=True)
    torch.cuda.synchronize()
    assert M1 is None and J2 is None
    assert np.array_equal(J1.double().cpu().numpy(), J) and np.array_equal(M2.double().cpu().numpy(), M)
    with pytest.raises(RuntimeError, match="bad arguments"):
        sim.jacobian_mass(0, jacobian=False, mass=False)
    with pytest.raises(ValueError, match="not one of this sim's 1 models"):
        sim.jacobian_mass(1)
