"""The env-step under HIP graph capture: a captured T-step loop replays bit-identically to eager steps."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2108_10470_amd import ags, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fp64", [True, False], ids=["fp64", "fp32"])
def test_captured_step_loop_replays_like_eager(fp64):
    env = W.env_humanoid()
    E, T = 256, 8
    p = W.SimParams()
    sim = ags.Sim([ags.Model(env)], [0] * E, p, device="cuda:0", fp64=fp64)
    root, dof = W.initial_state(env, E, 0)
    r0 = torch.tensor(root.reshape(-1, 13), dtype=torch.float32, device="cuda:0")
    d0 = torch.tensor(dof.reshape(-1, 2), dtype=torch.float32, device="cuda:0")
    acts = torch.tensor(W.actuation(env, E, 3 * T, 0).reshape(3 * T, -1), dtype=torch.float32, device="cuda:0")

    def eager(k0):
        for t in range(T):
            sim.bind(ags.DOF_ACTUATION, acts[k0 + t])
            sim.step()
        torch.cuda.synchronize()
        return sim.root_state.clone(), sim.dof_state.clone(), sim.contact_force.clone()

    # reference: eager steps from the start state (steps 0..T-1) and from the state they reach (T..2T-1)
    sim.root_state.copy_(r0); sim.dof_state.copy_(d0)
    ref1 = eager(0)
    ref2 = eager(T)
    # capture steps 0..T-1 (torch's capture stream is the current stream inside the context)
    sim.root_state.copy_(r0); sim.dof_state.copy_(d0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm the path on a side stream before capture
        sim.bind(ags.DOF_ACTUATION, acts[0])
        sim.step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for t in range(T):
            sim.bind(ags.DOF_ACTUATION, acts[t])
            sim.step()
    for rep in range(3):
        sim.root_state.copy_(r0); sim.dof_state.copy_(d0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (sim.root_state.clone(), sim.dof_state.clone(), sim.contact_force.clone())
        for a, b in zip(got, ref1):
            assert torch.equal(a, b), f"replay {rep} differs from the eager steps"
        # eager work between replays, continuing from the replayed state, must match the eager reference too
        cont = eager(T)
        for a, b in zip(cont, ref2):
            assert torch.equal(a, b), f"eager steps after replay {rep} differ"
