"""ags_rollout_backward_noalloc (segment buffers in the library's static device scratch) against
ags_rollout_backward (caller workspace) through the C ABI: identical adjoints, bit for bit, on two calls in
a row, the second with a smaller sim; and the size limit of the static scratch is refused."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2108_10470_amd import ags, workloads as W

pytestmark = pytest.mark.gpu

F32 = dict(dtype=torch.float32, device="cuda:0")


def _both(env, params, E, T, every, seed):
    """The rollout's reverse pass through both entry points from the same forward; returns both outputs."""
    L = ags.lib()
    sim = ags.Sim([ags.Model(env)], [0] * E, params, device="cuda:0", fp64=True)
    root, dof = W.initial_state(env, E, seed)
    acts = torch.tensor(W.actuation(env, E, T, seed).reshape(T, -1), **F32)
    sim.root_state.copy_(torch.tensor(root.reshape(-1, 13), **F32))
    sim.dof_state.copy_(torch.tensor(dof.reshape(-1, 2), **F32))
    n = ctypes.c_int64()
    ags._check(L.ags_rollout_state_size(sim.h, ctypes.byref(n)), "state_size")
    ckpt = torch.empty(((T + every - 1) // every, n.value), **F32)
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    ags._check(L.ags_rollout_forward(sim.h, T, every, ags.DOF_ACTUATION, P(acts), P(ckpt), sp), "forward")
    rng = np.random.default_rng(seed + 1)
    seed_root = torch.tensor(rng.standard_normal(sim.root_state.shape), **F32)
    seed_dof = torch.tensor(rng.standard_normal(sim.dof_state.shape), **F32)
    out = []
    for noalloc in (False, True):
        ra, da = seed_root.clone(), seed_dof.clone()
        aa = torch.full_like(acts, float("nan"))
        st = torch.full((E,), 7, dtype=torch.int32, device="cuda:0")
        if noalloc:
            rc = L.ags_rollout_backward_noalloc(sim.h, T, every, ags.DOF_ACTUATION, P(acts), P(ckpt), P(ra), P(da),
                                                P(aa), P(st), sp)
        else:
            nb = ctypes.c_int64()
            ags._check(L.ags_rollout_seg_bytes(sim.h, every, ctypes.byref(nb)), "seg_bytes")
            seg = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
            rc = L.ags_rollout_backward(sim.h, T, every, ags.DOF_ACTUATION, P(acts), P(ckpt), P(seg), P(ra), P(da),
                                        P(aa), P(st), sp)
        ags._check(rc, "backward")
        torch.cuda.synchronize()
        out.append((ra, da, aa, st))
    return out


@pytest.mark.parametrize("case", ["humanoid_then_smaller_ant"])
def test_noalloc_rollout_backward_equals_workspace_version(case):
    calls = [(W.as_f32(W.env_humanoid()), 64, 8, 4, 0), (W.as_f32(W.env_ant()), 16, 6, 3, 1)]
    for env, E, T, every, seed in calls:
        print("noalloc rollout backward:", env.name, "envs", E, "steps", T, "every", every, flush=True)
        ref, got = _both(env, W.params_f32(W.SimParams()), E, T, every, seed)
        for name, a, b in zip(("root_adj", "dof_adj", "act_adj", "status"), ref, got):
            assert torch.equal(a, b), (env.name, name)
        assert torch.isfinite(ref[2]).all() and float(ref[2].abs().max()) > 0
        assert int(ref[3].abs().sum()) == 0


def test_noalloc_rollout_backward_refuses_more_than_its_scratch():
    env = W.as_f32(W.env_humanoid())
    E, T = 4096, 13
    sim = ags.Sim([ags.Model(env)], [0] * E, W.params_f32(W.SimParams()), device="cuda:0", fp64=True)
    L = ags.lib()
    x = torch.zeros(1, **F32)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for every, ok in ((13, False), (12, True)):
        nb = ctypes.c_int64()
        ags._check(L.ags_rollout_seg_bytes(sim.h, every, ctypes.byref(nb)), "seg_bytes")
        assert (nb.value <= 64 << 20) == ok, (every, nb.value)
    rc = L.ags_rollout_backward_noalloc(sim.h, T, 13, ags.DOF_ACTUATION, P(x), P(x), P(x), P(x), P(x), None, sp)
    assert rc != 0 and b"static scratch" in L.ags_last_error()
