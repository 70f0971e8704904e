"""Python binding of libags (ctypes): argument marshalling only.

Every step of the physics runs in the HIP kernels of libags.so; PyTorch supplies device memory and
streams.  The library must be built (``python -m paper_2108_10470_amd.build``); importing this
module fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, List, Optional, Sequence

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libags.so")

JOINT = {"free": 0, "fixed": 1, "revolute": 2, "prismatic": 3}
SHAPE = {"sphere": 0, "capsule": 1, "box": 2}

ROOT_STATE, DOF_STATE, DOF_ACTUATION, DOF_POS_TARGET, DOF_VEL_TARGET, NET_CONTACT_FORCE, DOF_FORCE, \
    DEBUG_QDD_FREE, DEBUG_ROW_COUNT, DEBUG_ROW_KEY, DEBUG_ROW_LAMBDA, DEBUG_PHASE_CYCLES, DEBUG_ADJ_CYCLES, \
    RIGID_BODY_STATE, ENV_STATUS, BODY_MASS_SCALE, DOF_STIFFNESS, DOF_DAMPING, DOF_LIMITS, ENV_FRICTION, \
    ENV_GRAVITY, NUM_TENSORS = range(22)
PHASES = ["controls", "forward", "inward", "outward", "vstar", "narrow", "rows", "responses", "pgs", "outputs"]


class LinkDesc(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_int32), ("joint", ctypes.c_int32), ("anchor", ctypes.c_float * 3),
                ("axis", ctypes.c_float * 3), ("lower", ctypes.c_float), ("upper", ctypes.c_float),
                ("kp", ctypes.c_float), ("kd", ctypes.c_float), ("armature", ctypes.c_float), ("mass", ctypes.c_float)]


class ShapeDesc(ctypes.Structure):
    _fields_ = [("link", ctypes.c_int32), ("kind", ctypes.c_int32), ("p0", ctypes.c_float * 3),
                ("p1", ctypes.c_float * 3), ("radius", ctypes.c_float), ("half", ctypes.c_float * 3),
                ("density", ctypes.c_float)]


class ActorDesc(ctypes.Structure):
    _fields_ = [("n_links", ctypes.c_int32), ("n_shapes", ctypes.c_int32), ("links", ctypes.POINTER(LinkDesc)),
                ("shapes", ctypes.POINTER(ShapeDesc))]


class PairDesc(ctypes.Structure):
    _fields_ = [("a_actor", ctypes.c_int32), ("a_shape", ctypes.c_int32), ("b_actor", ctypes.c_int32),
                ("b_shape", ctypes.c_int32)]


class TendonDesc(ctypes.Structure):
    _fields_ = [("actor", ctypes.c_int32), ("n_joints", ctypes.c_int32), ("link", ctypes.POINTER(ctypes.c_int32)),
                ("parent", ctypes.POINTER(ctypes.c_int32)), ("coef", ctypes.POINTER(ctypes.c_float)),
                ("stiffness", ctypes.c_float), ("damping", ctypes.c_float), ("rest_length", ctypes.c_float),
                ("lower", ctypes.c_float), ("upper", ctypes.c_float), ("limit_stiffness", ctypes.c_float)]


class ModelInfo(ctypes.Structure):
    _fields_ = [("n_actors", ctypes.c_int32), ("n_links", ctypes.c_int32), ("n_dof", ctypes.c_int32),
                ("n_v", ctypes.c_int32), ("n_slots", ctypes.c_int32), ("max_rows", ctypes.c_int32)]


class SimParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("substeps", ctypes.c_int32), ("gravity", ctypes.c_float * 3),
                ("pgs_iters", ctypes.c_int32), ("mu", ctypes.c_float), ("baumgarte", ctypes.c_float),
                ("contact_margin", ctypes.c_float), ("limit_margin_rev", ctypes.c_float),
                ("limit_margin_pri", ctypes.c_float), ("compute_fp64", ctypes.c_int32),
                ("lanes_per_env", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("adjoint_precision", ctypes.c_int32), ("solver", ctypes.c_int32),
                ("adjoint_max_rows", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded libags; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libags.so not built ({LIB_PATH}); run python -m paper_2108_10470_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
        L.ags_last_error.restype = ctypes.c_char_p
        L.ags_model_create.argtypes = [ctypes.POINTER(ActorDesc), i32, ctypes.POINTER(PairDesc), i32, ctypes.POINTER(vp)]
        L.ags_model_destroy.argtypes = [vp]
        L.ags_model_add_tendons.argtypes = [vp, ctypes.POINTER(TendonDesc), i32]
        L.ags_model_get_info.argtypes = [vp, ctypes.POINTER(ModelInfo)]
        L.ags_model_mass_props.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(ctypes.c_float)]
        L.ags_sim_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_int32), i32,
                                     ctypes.POINTER(SimParams), ctypes.POINTER(vp)]
        L.ags_sim_destroy.argtypes = [vp]
        L.ags_sim_tensor_shape.argtypes = [vp, i32, i64p, i64p]
        L.ags_sim_bind.argtypes = [vp, i32, vp]
        L.ags_sim_step.argtypes = [vp, vp]
        L.ags_sim_set_root_state_indexed.argtypes = [vp, vp, vp, i32, vp]
        L.ags_sim_set_dof_state_indexed.argtypes = [vp, vp, vp, i32, vp]
        L.ags_sim_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ags_rollout_state_size.argtypes = [vp, i64p]
        L.ags_rollout_seg_bytes.argtypes = [vp, i32, i64p]
        L.ags_autotune.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_int32), i32, ctypes.POINTER(SimParams),
                                   vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float), vp]
        L.ags_rollout_forward.argtypes = [vp, i32, i32, i32, vp, vp, vp]
        L.ags_rollout_backward.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ags_rollout_backward_noalloc.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.ags_rollout_tape_bytes.argtypes = [vp, i32, i64p]
        L.ags_sim_jacobian_mass.argtypes = [vp, i32, vp, vp, vp]
        L.ags_rollout_forward_tape.argtypes = [vp, i32, i32, vp, vp, vp]
        L.ags_rollout_backward_tape.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
        _lib = L
    return _lib


EXPORTED = ["ags_last_error", "ags_model_create", "ags_model_destroy", "ags_model_get_info", "ags_model_mass_props",
            "ags_sim_create", "ags_sim_destroy", "ags_sim_tensor_shape", "ags_sim_bind", "ags_sim_step",
            "ags_sim_set_root_state_indexed", "ags_sim_set_dof_state_indexed", "ags_sim_step_backward",
            "ags_rollout_state_size", "ags_rollout_forward", "ags_rollout_backward", "ags_autotune",
            "ags_rollout_seg_bytes", "ags_rollout_tape_bytes", "ags_rollout_forward_tape", "ags_rollout_backward_tape",
            "ags_sim_jacobian_mass", "ags_model_add_tendons", "ags_rollout_backward_noalloc"]


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed ({rc}): {lib().ags_last_error().decode()}")


def _f3(v):
    return (ctypes.c_float * 3)(*[float(x) for x in v])


class Model:
    """One compiled environment template (actors + collision pairs) from a workloads.EnvSpec."""

    def __init__(self, env):
        self.spec = env
        keep = []
        actors = (ActorDesc * len(env.actors))()
        shape_index = {}
        for ai, a in enumerate(env.actors):
            links = (LinkDesc * len(a.links))()
            shapes = []
            for li, l in enumerate(a.links):
                links[li] = LinkDesc(l.parent, JOINT[l.joint], _f3(l.anchor), _f3(l.axis), l.lower, l.upper, l.kp, l.kd,
                                     l.armature, l.mass)
                for si, s in enumerate(l.shapes):
                    shape_index[(ai, li, si)] = len(shapes)
                    shapes.append(ShapeDesc(li, SHAPE[s.kind], _f3(s.p0), _f3(s.p1), s.radius, _f3(s.half), s.density))
            sarr = (ShapeDesc * max(1, len(shapes)))(*shapes)
            keep += [links, sarr]
            actors[ai] = ActorDesc(len(a.links), len(shapes), links, sarr)
        pairs = (PairDesc * max(1, len(env.pairs)))()
        for k, p in enumerate(env.pairs):
            pairs[k] = PairDesc(p.a_actor, shape_index[(p.a_actor, p.a_link, p.a_shape)], p.b_actor,
                                shape_index[(p.b_actor, p.b_link, p.b_shape)] if p.b_actor >= 0 else -1)
        h = ctypes.c_void_p()
        _check(lib().ags_model_create(actors, len(env.actors), pairs, len(env.pairs), ctypes.byref(h)), "ags_model_create")
        self.h = h
        tds = []
        for ai, a in enumerate(env.actors):
            for t in a.tendons:
                n = len(t.links)
                arrs = ((ctypes.c_int32 * n)(*t.links), (ctypes.c_int32 * n)(*t.parents), (ctypes.c_float * n)(*t.coefs))
                keep.append(arrs)
                tds.append(TendonDesc(ai, n, arrs[0], arrs[1], arrs[2], t.stiffness, t.damping, t.rest_length,
                                      t.lower, t.upper, t.limit_stiffness))
        if tds:
            _check(lib().ags_model_add_tendons(h, (TendonDesc * len(tds))(*tds), len(tds)), "ags_model_add_tendons")
        info = ModelInfo()
        _check(lib().ags_model_get_info(h, ctypes.byref(info)), "ags_model_get_info")
        self.info = info

    def mass_props(self):
        n = self.info.n_links
        m = (ctypes.c_float * n)()
        c = (ctypes.c_float * (3 * n))()
        I = (ctypes.c_float * (9 * n))()
        _check(lib().ags_model_mass_props(self.h, m, c, I), "ags_model_mass_props")
        import numpy as np
        return (np.array(m[:]), np.array(c[:]).reshape(n, 3), np.array(I[:]).reshape(n, 3, 3))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ags_model_destroy(self.h)
            self.h = None


def sim_params(p, fp64: bool = False, lanes_per_env: int = 0, persistent: bool = False,
               adjoint_precision: int = 0, adjoint_max_rows: int = 0) -> SimParams:
    return SimParams(p.dt, p.substeps, _f3(p.gravity), p.pgs_iters, p.mu, p.baumgarte, p.contact_margin,
                     p.limit_margin_rev, p.limit_margin_pri, 1 if fp64 else 0, lanes_per_env, 1 if persistent else 0,
                     adjoint_precision, int(getattr(p, "solver", 0)), adjoint_max_rows)


class Sim:
    """A batch of environments with its state and control tensors allocated by torch on `device`."""

    def __init__(self, models: Sequence[Model], env_model: Sequence[int], params, device="cuda:0",
                 debug: bool = False, pd: bool = False, fp64: bool = False, phase_cycles: bool = False,
                 lanes_per_env: int = 0, persistent: bool = False, adjoint_precision: int = 0,
                 rigid_body_state: bool = False, status: bool = False, adjoint_max_rows: int = 0):
        self.models = list(models)
        self.env_model = [int(x) for x in env_model]
        self.params = params
        self.device = torch.device(device)
        self.n_envs = len(env_model)
        handles = (ctypes.c_void_p * len(self.models))(*[m.h for m in self.models])
        ids = (ctypes.c_int32 * self.n_envs)(*[int(x) for x in env_model])
        h = ctypes.c_void_p()
        self._p = sim_params(params, fp64, lanes_per_env, persistent, adjoint_precision, adjoint_max_rows)
        _check(lib().ags_sim_create(handles, len(self.models), ids, self.n_envs, ctypes.byref(self._p), ctypes.byref(h)),
               "ags_sim_create")
        self.h = h
        self.tensors: Dict[int, torch.Tensor] = {}
        shapes = {}
        for w in range(NUM_TENSORS):
            r, c = ctypes.c_int64(), ctypes.c_int64()
            _check(lib().ags_sim_tensor_shape(h, w, ctypes.byref(r), ctypes.byref(c)), "ags_sim_tensor_shape")
            shapes[w] = (r.value, c.value)
        self.shapes = shapes
        f32 = dict(dtype=torch.float32, device=self.device)
        self.root_state = self._alloc(ROOT_STATE, torch.zeros(shapes[ROOT_STATE], **f32))
        self.dof_state = self._alloc(DOF_STATE, torch.zeros(shapes[DOF_STATE], **f32))
        self.actuation = self._alloc(DOF_ACTUATION, torch.zeros(shapes[DOF_ACTUATION][0], **f32))
        self.contact_force = self._alloc(NET_CONTACT_FORCE, torch.zeros(shapes[NET_CONTACT_FORCE], **f32))
        self.dof_force = self._alloc(DOF_FORCE, torch.zeros(shapes[DOF_FORCE][0], **f32))
        if rigid_body_state:
            self.rb_state = self._alloc(RIGID_BODY_STATE, torch.zeros(shapes[RIGID_BODY_STATE], **f32))
        if status:
            self.env_status = self._alloc(ENV_STATUS, torch.zeros(shapes[ENV_STATUS][0], dtype=torch.int32,
                                                                  device=self.device))
        if pd:
            self.pos_target = self._alloc(DOF_POS_TARGET, torch.zeros(shapes[DOF_POS_TARGET][0], **f32))
            self.vel_target = self._alloc(DOF_VEL_TARGET, torch.zeros(shapes[DOF_VEL_TARGET][0], **f32))
        if phase_cycles:
            self.dbg_cycles = self._alloc(DEBUG_PHASE_CYCLES, torch.zeros(shapes[DEBUG_PHASE_CYCLES], dtype=torch.int64,
                                                                          device=self.device))
        if debug:
            self.dbg_qdd = self._alloc(DEBUG_QDD_FREE, torch.zeros(shapes[DEBUG_QDD_FREE], **f32))
            self.dbg_rc = self._alloc(DEBUG_ROW_COUNT, torch.zeros(shapes[DEBUG_ROW_COUNT], dtype=torch.int32, device=self.device))
            self.dbg_key = self._alloc(DEBUG_ROW_KEY, torch.full(shapes[DEBUG_ROW_KEY], -1, dtype=torch.int32, device=self.device))
            self.dbg_lam = self._alloc(DEBUG_ROW_LAMBDA, torch.zeros(shapes[DEBUG_ROW_LAMBDA], **f32))

    def _alloc(self, which: int, t: torch.Tensor) -> torch.Tensor:
        self.bind(which, t)
        return t

    def bind(self, which: int, t: Optional[torch.Tensor]):
        if t is not None:
            assert t.is_contiguous() and t.device == self.device
        self.tensors[which] = t
        _check(lib().ags_sim_bind(self.h, which, ctypes.c_void_p(t.data_ptr() if t is not None else 0)), "ags_sim_bind")

    def step(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib().ags_sim_step(self.h, ctypes.c_void_p(s.cuda_stream)), "ags_sim_step")

    def _dev_f32(self, t: torch.Tensor, shape, what: str):
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what}: expected a contiguous float32 tensor of shape {tuple(shape)} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return ctypes.c_void_p(t.data_ptr())

    def step_backward(self, root_state: torch.Tensor, dof_state: torch.Tensor, actuation: torch.Tensor,
                      root_adj: torch.Tensor, dof_adj: torch.Tensor, act_adj: torch.Tensor,
                      status: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None):
        """Adjoint of one env-step started from (root_state, dof_state) with `actuation`: root_adj/dof_adj
        hold dL/d(state after) on entry and dL/d(state before) on return; act_adj receives dL/d actuation."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        rs, ds, na = self.shapes[ROOT_STATE], self.shapes[DOF_STATE], self.shapes[DOF_ACTUATION][0]
        args = [self._dev_f32(root_state, rs, "root_state"), self._dev_f32(dof_state, ds, "dof_state"),
                self._dev_f32(actuation, (na,), "actuation"), self._dev_f32(root_adj, rs, "root_adj"),
                self._dev_f32(dof_adj, ds, "dof_adj"), self._dev_f32(act_adj, (na,), "act_adj")]
        st = ctypes.c_void_p(0)
        if status is not None:
            if status.dtype != torch.int32 or status.device != self.device or status.numel() != self.n_envs:
                raise ValueError("status: expected an int32 tensor with one entry per environment")
            st = ctypes.c_void_p(status.data_ptr())
        _check(lib().ags_sim_step_backward(self.h, *args, st, ctypes.c_void_p(s.cuda_stream)), "ags_sim_step_backward")

    def set_properties(self, mass_scale=None, stiffness=None, damping=None, limits=None, friction=None,
                       gravity=None):
        """Bind per-env property tensors (domain randomization; see ags.h): (N_B,) link mass factors, (N_D,)
        drive kp and kd, (N_D, 2) limits, (E,) friction, (E, 3) gravity.  A None argument leaves that
        property as it is; pass a tensor to replace the model's value, or call unbind_properties()."""
        for which, t, shape in ((BODY_MASS_SCALE, mass_scale, (self.shapes[BODY_MASS_SCALE][0],)),
                                (DOF_STIFFNESS, stiffness, (self.shapes[DOF_STIFFNESS][0],)),
                                (DOF_DAMPING, damping, (self.shapes[DOF_DAMPING][0],)),
                                (DOF_LIMITS, limits, self.shapes[DOF_LIMITS]),
                                (ENV_FRICTION, friction, (self.n_envs,)),
                                (ENV_GRAVITY, gravity, (self.n_envs, 3))):
            if t is not None:
                self._dev_f32(t, shape, "property tensor")
                self.bind(which, t)

    def unbind_properties(self):
        for which in (BODY_MASS_SCALE, DOF_STIFFNESS, DOF_DAMPING, DOF_LIMITS, ENV_FRICTION, ENV_GRAVITY):
            lib().ags_sim_bind(self.h, which, ctypes.c_void_p(0))
            self.tensors.pop(which, None)

    def jacobian_mass(self, model: int = 0, jacobian: bool = True, mass: bool = True,
                      stream: Optional[torch.cuda.Stream] = None):
        """Jacobian (n, n_links, 6, n_v) and generalized mass matrix (n, n_v, n_v) tensors of the n envs
        that use models[model], in env order, at the bound state (ags_sim_jacobian_mass); None for an
        output not asked for."""
        if not 0 <= model < len(self.models):
            raise ValueError(f"jacobian_mass: model {model} is not one of this sim's {len(self.models)} models")
        n = sum(1 for m in self.env_model if m == model)
        info = self.models[model].info
        f32 = dict(dtype=torch.float32, device=self.device)
        J = torch.empty((n, info.n_links, 6, info.n_v), **f32) if jacobian else None
        M = torch.empty((n, info.n_v, info.n_v), **f32) if mass else None
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(lib().ags_sim_jacobian_mass(self.h, model, ctypes.c_void_p(J.data_ptr() if J is not None else 0),
                                           ctypes.c_void_p(M.data_ptr() if M is not None else 0),
                                           ctypes.c_void_p(s.cuda_stream)), "ags_sim_jacobian_mass")
        return J, M

    def set_root_state_indexed(self, src: torch.Tensor, actor_idx: Optional[torch.Tensor] = None):
        s = torch.cuda.current_stream(self.device)
        n = 0 if actor_idx is None else actor_idx.numel()
        if actor_idx is None:
            n = self.shapes[ROOT_STATE][0]
        _check(lib().ags_sim_set_root_state_indexed(self.h, ctypes.c_void_p(src.data_ptr()),
                                                    ctypes.c_void_p(actor_idx.data_ptr() if actor_idx is not None else 0),
                                                    n, ctypes.c_void_p(s.cuda_stream)), "ags_sim_set_root_state_indexed")

    def set_dof_state_indexed(self, src: torch.Tensor, actor_idx: Optional[torch.Tensor] = None):
        s = torch.cuda.current_stream(self.device)
        n = self.shapes[ROOT_STATE][0] if actor_idx is None else actor_idx.numel()
        _check(lib().ags_sim_set_dof_state_indexed(self.h, ctypes.c_void_p(src.data_ptr()),
                                                   ctypes.c_void_p(actor_idx.data_ptr() if actor_idx is not None else 0),
                                                   n, ctypes.c_void_p(s.cuda_stream)), "ags_sim_set_dof_state_indexed")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ags_sim_destroy(self.h)
            self.h = None


class Rollout(torch.autograd.Function):
    """Differentiable rollout: final (root_state, dof_state) after T env-steps of `sim` from (root0, dof0)
    with actions (T, N_D).  With every >= 1 the forward pass keeps the state every `every` steps and the
    backward pass recomputes each segment from its checkpoint (ags_rollout_forward / ags_rollout_backward);
    with every = 0 the forward pass stores the whole tape and the backward pass recomputes nothing
    (ags_rollout_forward_tape / ags_rollout_backward_tape).  Either way the adjoint of every step runs in
    reverse; gradients flow to the actions and the initial state."""

    @staticmethod
    def forward(ctx, actions, root0, dof0, sim, every, control=DOF_ACTUATION):
        T = actions.shape[0]
        actions = actions.contiguous()
        sim._dev_f32(actions, (T, sim.shapes[DOF_ACTUATION][0]), "actions")
        if every < 0:
            raise ValueError("every must be >= 1 (checkpoints) or 0 (stored tape)")
        sim.root_state.copy_(root0)
        sim.dof_state.copy_(dof0)
        n = ctypes.c_int64()
        s = torch.cuda.current_stream(sim.device)
        if every == 0:
            _check(lib().ags_rollout_tape_bytes(sim.h, T, ctypes.byref(n)), "ags_rollout_tape_bytes")
            ckpt = torch.empty(n.value, dtype=torch.uint8, device=sim.device)
            _check(lib().ags_rollout_forward_tape(sim.h, T, control, ctypes.c_void_p(actions.data_ptr()),
                                                  ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(s.cuda_stream)),
                   "ags_rollout_forward_tape")
        else:
            _check(lib().ags_rollout_state_size(sim.h, ctypes.byref(n)), "ags_rollout_state_size")
            ckpt = torch.empty(((T + every - 1) // every, n.value), dtype=torch.float32, device=sim.device)
            _check(lib().ags_rollout_forward(sim.h, T, every, control, ctypes.c_void_p(actions.data_ptr()),
                                             ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(s.cuda_stream)),
                   "ags_rollout_forward")
        ctx.save_for_backward(actions, ckpt)
        ctx.sim, ctx.every, ctx.state_words, ctx.control = sim, every, n.value, control
        return sim.root_state.clone(), sim.dof_state.clone()

    @staticmethod
    def backward(ctx, g_root, g_dof):
        actions, ckpt = ctx.saved_tensors
        sim, every = ctx.sim, ctx.every
        T = actions.shape[0]
        root_adj = (g_root if g_root is not None else torch.zeros_like(sim.root_state)).float().contiguous().clone()
        dof_adj = (g_dof if g_dof is not None else torch.zeros_like(sim.dof_state)).float().contiguous().clone()
        act_adj = torch.empty_like(actions)
        status = torch.zeros(sim.n_envs, dtype=torch.int32, device=sim.device)
        s = torch.cuda.current_stream(sim.device)
        if every == 0:
            _check(lib().ags_rollout_backward_tape(sim.h, T, ctx.control, ctypes.c_void_p(actions.data_ptr()),
                                                   ctypes.c_void_p(ckpt.data_ptr()),
                                                   ctypes.c_void_p(root_adj.data_ptr()),
                                                   ctypes.c_void_p(dof_adj.data_ptr()),
                                                   ctypes.c_void_p(act_adj.data_ptr()),
                                                   ctypes.c_void_p(status.data_ptr()),
                                                   ctypes.c_void_p(s.cuda_stream)), "ags_rollout_backward_tape")
        else:
            nb = ctypes.c_int64()
            _check(lib().ags_rollout_seg_bytes(sim.h, every, ctypes.byref(nb)), "ags_rollout_seg_bytes")
            seg = torch.empty(nb.value, dtype=torch.uint8, device=sim.device)
            _check(lib().ags_rollout_backward(sim.h, T, every, ctx.control, ctypes.c_void_p(actions.data_ptr()),
                                              ctypes.c_void_p(ckpt.data_ptr()), ctypes.c_void_p(seg.data_ptr()),
                                              ctypes.c_void_p(root_adj.data_ptr()), ctypes.c_void_p(dof_adj.data_ptr()),
                                              ctypes.c_void_p(act_adj.data_ptr()), ctypes.c_void_p(status.data_ptr()),
                                              ctypes.c_void_p(s.cuda_stream)), "ags_rollout_backward")
        sim.last_rollout_status = status
        bad = int((status != 0).sum())
        if bad:
            raise RuntimeError(f"adjoint: {bad} environments exceeded the adjoint's row capacity at some step "
                               f"(adjoint_max_rows, default 64 rows per substep)")
        return act_adj, root_adj, dof_adj, None, None, None


def rollout(sim: "Sim", actions: torch.Tensor, root0: torch.Tensor, dof0: torch.Tensor, every: int = 16,
            control: int = DOF_ACTUATION):
    """Differentiable T-step rollout (see Rollout): checkpoints every `every` steps, or the whole tape
    stored with every = 0; `control` selects what actions[t] drives: the actuation (DOF_ACTUATION) or the
    PD position targets (DOF_POS_TARGET)."""
    return Rollout.apply(actions, root0, dof0, sim, every, control)


def autotune(models: Sequence[Model], env_model: Sequence[int], params, root_state: torch.Tensor,
             dof_state: torch.Tensor, actuation: torch.Tensor, fp64: bool = False, n_steps: int = 10):
    """The fastest (lanes_per_env, persistent) mapping for this batch (ags_autotune): returns
    (lanes_per_env, persistent, ms per env-step)."""
    handles = (ctypes.c_void_p * len(models))(*[m.h for m in models])
    ids = (ctypes.c_int32 * len(env_model))(*[int(x) for x in env_model])
    sp = sim_params(params, fp64)
    ms = ctypes.c_float()
    s = torch.cuda.current_stream(root_state.device)
    n_a = sum(models[m].info.n_actors for m in env_model)
    n_d = sum(models[m].info.n_dof for m in env_model)
    for t, n, what in ((root_state, 13 * n_a, "root_state"), (dof_state, 2 * n_d, "dof_state"), (actuation, n_d, "actuation")):
        if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda or t.numel() != n:
            raise ValueError(f"autotune: {what} must be a contiguous float32 device tensor of {n} elements")
    _check(lib().ags_autotune(handles, len(models), ids, len(env_model), ctypes.byref(sp),
                              ctypes.c_void_p(root_state.data_ptr()), ctypes.c_void_p(dof_state.data_ptr()),
                              ctypes.c_void_p(actuation.data_ptr()), n_steps, ctypes.byref(ms),
                              ctypes.c_void_p(s.cuda_stream)), "ags_autotune")
    return sp.lanes_per_env, bool(sp.persistent), ms.value
