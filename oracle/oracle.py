"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and bench.py's CPU-baseline
leg.  The product path (paper_2108_10470_amd) never imports this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

L_COLS = 15
S_COLS = 14
P_COLS = 13
_JOINT = {"free": 0, "fixed": 1, "revolute": 2, "prismatic": 3}
_KIND = {"sphere": 0, "capsule": 1, "box": 2}

NEAR_CONTACT, NEAR_LIMIT, NEAR_GEOM, NEAR_SKIP, NEAR_TANGENT, NEAR_CLAMP = 1, 2, 4, 8, 16, 32
# the bits that mark a possible jump of the step's value (a row that may or may not exist, an ambiguous
# geometric choice); NEAR_CLAMP marks only a switch of its derivative (the projection is continuous)
NEAR_VALUE = NEAR_CONTACT | NEAR_LIMIT | NEAR_GEOM | NEAR_SKIP | NEAR_TANGENT

# guard widths of the mode-switch test: an env-substep is "near a switch" when a contact
# activation test lies within GUARD_C metres, or a limit activation test within GUARD_L rad (m),
# of its threshold
GUARD_C = 1e-5
GUARD_L = 1e-5


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "oracle.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-o", tmp, src])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_env_create.restype = ctypes.c_void_p
        L.orc_env_create.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, ip,
                                     ctypes.c_char_p, ctypes.c_int]
        L.orc_env_destroy.argtypes = [ctypes.c_void_p]
        L.orc_env_sizes.argtypes = [ctypes.c_void_p, ip]
        L.orc_env_set_tendons.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_mass_props.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_fk.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        L.orc_body_states.argtypes = [ctypes.c_void_p, dp, dp, dp]
        L.orc_dynamics.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_dynamics.restype = ctypes.c_int
        L.orc_slots.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, ip, ip]
        L.orc_slots.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.c_void_p, dp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int, ip,
                               ip, dp, dp, dp, dp, ip, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
        L.orc_step.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def env_tables(env):
    """Oracle tables (its own layout) from a workloads.EnvSpec."""
    links, shapes, pairs = [], [], []
    shape_row = {}
    for ai, a in enumerate(env.actors):
        for li, l in enumerate(a.links):
            row = np.zeros(L_COLS)
            row[0] = ai
            row[1] = l.parent
            row[2] = _JOINT[l.joint]
            row[3:6] = l.anchor
            row[6:9] = l.axis
            row[9], row[10] = l.lower, l.upper
            row[11], row[12], row[13], row[14] = l.kp, l.kd, l.armature, l.mass
            links.append(row)
            for si, s in enumerate(l.shapes):
                srow = np.zeros(S_COLS)
                srow[0], srow[1], srow[2] = ai, li, _KIND[s.kind]
                srow[3:6] = s.p0
                srow[6:9] = s.p1
                srow[9] = s.radius
                srow[10:13] = s.half
                srow[13] = s.density
                shape_row[(ai, li, si)] = len(shapes)
                shapes.append(srow)
    for p in env.pairs:
        a = shape_row[(p.a_actor, p.a_link, p.a_shape)]
        b = shape_row[(p.b_actor, p.b_link, p.b_shape)] if p.b_actor >= 0 else -1
        pairs.append([p.a_actor, p.a_link, a, p.b_actor, p.b_link, b])
    return (np.ascontiguousarray(np.array(links, dtype=np.float64)),
            np.ascontiguousarray(np.array(shapes, dtype=np.float64).reshape(-1, S_COLS)),
            np.ascontiguousarray(np.array(pairs, dtype=np.int32).reshape(-1, 6)))


def params_vector(p, guard_c=GUARD_C, guard_l=GUARD_L):
    return np.array([p.dt, p.substeps, *p.gravity, p.pgs_iters, p.mu, p.baumgarte, p.contact_margin,
                     p.limit_margin_rev, p.limit_margin_pri, guard_c, guard_l, getattr(p, "solver", 0)],
                    dtype=np.float64)


class OracleEnv:
    """One env template (actors + pairs) evaluated in FP64 on the CPU."""

    def __init__(self, env):
        self.spec = env
        links, shapes, pairs = env_tables(env)
        err = ctypes.create_string_buffer(256)
        h = lib().orc_env_create(env.n_actors, len(links), _dp(links), len(shapes), _dp(shapes), len(pairs),
                                 _ip(pairs), err, 256)
        if not h:
            raise ValueError("oracle: " + err.value.decode())
        self.h = h
        tparams, tjoints = [], []
        dof_off = 0
        for a in env.actors:
            for t in a.tendons:
                tid = len(tparams)
                tparams.append([t.stiffness, t.damping, t.rest_length, t.lower, t.upper, t.limit_stiffness])
                for link, par, c in zip(t.links, t.parents, t.coefs):
                    tjoints.append([tid, dof_off + link - 1, par, c])
            dof_off += a.n_dof
        if tparams:
            tp = np.ascontiguousarray(tparams, dtype=np.float64)
            tj = np.ascontiguousarray(tjoints, dtype=np.float64)
            lib().orc_env_set_tendons(h, len(tparams), _dp(tp), len(tjoints), _dp(tj))
        s = np.zeros(6, dtype=np.int32)
        lib().orc_env_sizes(h, _ip(s))
        self.n_dof, self.n_v, self.n_bodies, self.n_actors, self.max_rows, self.n_slots = map(int, s)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_env_destroy(self.h)
            self.h = None

    def mass_props(self):
        m = np.zeros(self.n_bodies)
        c = np.zeros((self.n_bodies, 3))
        I = np.zeros((self.n_bodies, 3, 3))
        lib().orc_mass_props(self.h, _dp(m), _dp(c), _dp(I))
        return m, c, I

    def fk(self, root, dof):
        root = np.ascontiguousarray(root, dtype=np.float64)
        dof = np.ascontiguousarray(dof, dtype=np.float64)
        R = np.zeros((self.n_bodies, 3, 3))
        p = np.zeros((self.n_bodies, 3))
        lib().orc_fk(self.h, _dp(root), _dp(dof), _dp(R), _dp(p))
        return R, p

    def body_states(self, root, dof):
        """Per body: link-frame origin (3), rotation to world (3 x 3), velocity of the origin (3) and
        angular velocity (3), world frame; one env (root (A, 13), dof (D, 2))."""
        root = np.ascontiguousarray(root, dtype=np.float64)
        dof = np.ascontiguousarray(dof, dtype=np.float64)
        out = np.zeros((self.n_bodies, 18))
        lib().orc_body_states(self.h, _dp(root), _dp(dof), _dp(out))
        return out[:, :3], out[:, 3:12].reshape(-1, 3, 3), out[:, 12:15], out[:, 15:18]

    def set_velocity(self, root, dof, qd):
        """Copies of one env's (root (A, 13), dof (D, 2)) with the generalized velocity qd (n_v) written in:
        per actor, a free root's world COM velocity and angular velocity (root columns 7-12), then the
        actor's joint rates."""
        root = np.array(root, dtype=np.float64)
        dof = np.array(dof, dtype=np.float64)
        c = j = 0
        for ai, a in enumerate(self.spec.actors):
            if not a.fixed_base:
                root[ai, 7:13] = qd[c:c + 6]
                c += 6
            dof[j:j + a.n_dof, 1] = qd[c:c + a.n_dof]
            c += a.n_dof
            j += a.n_dof
        return root, dof

    def jacobian(self, root, dof):
        """Jacobian tensor of one env (Section 2.3, Table 1), (n_bodies, 6, n_v): the rigid-body velocities
        (world velocity of each link origin, then its world angular velocity) are linear in the generalized
        velocity, and column k is their value at the unit generalized velocity e_k."""
        nv = self.n_v
        J = np.zeros((self.n_bodies, 6, nv))
        for k in range(nv):
            e = np.zeros(nv)
            e[k] = 1.0
            _, _, v, w = self.body_states(*self.set_velocity(root, dof, e))
            J[:, 0:3, k] = v
            J[:, 3:6, k] = w
        return J

    def mass_matrix(self, root, dof):
        """Generalized mass matrix of one env (Table 1), (n_v, n_v): the joint-space inertia M(q) of CRBA,
        without armature."""
        from types import SimpleNamespace
        p = SimpleNamespace(dt=1.0, substeps=1, gravity=(0.0, 0.0, 0.0), pgs_iters=0, mu=0.0, baumgarte=0.0,
                            contact_margin=0.0, limit_margin_rev=0.0, limit_margin_pri=0.0)
        return self.dynamics(p, root, dof, np.zeros(self.n_v))[0]

    def dynamics(self, params, root, dof, tau):
        root = np.ascontiguousarray(root, dtype=np.float64)
        dof = np.ascontiguousarray(dof, dtype=np.float64)
        tau = np.ascontiguousarray(tau, dtype=np.float64)
        nv = self.n_v
        M = np.zeros((nv, nv))
        C = np.zeros(nv)
        q1 = np.zeros(nv)
        q2 = np.zeros(nv)
        rc = lib().orc_dynamics(self.h, _dp(params_vector(params)), _dp(root), _dp(dof), _dp(tau), _dp(M), _dp(C),
                                _dp(q1), _dp(q2))
        if rc != 0:
            raise ValueError("oracle: mass matrix not positive definite")
        return M, C, q1, q2

    def slots(self, root, dof):
        root = np.ascontiguousarray(root, dtype=np.float64)
        dof = np.ascontiguousarray(dof, dtype=np.float64)
        n = max(self.n_slots, 1)
        phi = np.zeros(n)
        nrm = np.zeros((n, 3))
        pt = np.zeros((n, 3))
        ba = np.zeros(n, dtype=np.int32)
        bb = np.zeros(n, dtype=np.int32)
        k = lib().orc_slots(self.h, _dp(root), _dp(dof), _dp(phi), _dp(nrm), _dp(pt), _ip(ba), _ip(bb))
        return phi[:k], nrm[:k], pt[:k], ba[:k], bb[:k]

    def step(self, params, root, dof, act, pos_tgt=None, vel_tgt=None, n_threads=None, r_cap=None,
             guard_c=GUARD_C, guard_l=GUARD_L):
        """One env-step for a batch: root (E, A, 13), dof (E, D, 2), controls (E, D)."""
        root = np.ascontiguousarray(root, dtype=np.float64)
        dof = np.ascontiguousarray(dof, dtype=np.float64)
        E = root.shape[0]
        act = np.ascontiguousarray(np.broadcast_to(act, (E, self.n_dof)), dtype=np.float64)
        pt = None if pos_tgt is None else np.ascontiguousarray(np.broadcast_to(pos_tgt, (E, self.n_dof)), dtype=np.float64)
        vt = None if vel_tgt is None else np.ascontiguousarray(np.broadcast_to(vel_tgt, (E, self.n_dof)), dtype=np.float64)
        S = params.substeps
        r_cap = r_cap or max(self.max_rows, 1)
        out = dict(
            root=np.zeros_like(root), dof=np.zeros_like(dof), qdd_free=np.zeros((E, S, self.n_v)),
            row_count=np.zeros((E, S), dtype=np.int32), row_key=np.full((E, S, r_cap), -1, dtype=np.int32),
            row_lambda=np.zeros((E, S, r_cap)), contact_force=np.zeros((E, self.n_bodies, 3)),
            contact_scale=np.zeros((E, self.n_bodies, 2)),
            dof_force=np.zeros((E, self.n_dof)), near=np.zeros((E, S), dtype=np.int32),
            mode=np.zeros(E, dtype=np.uint64))
        nt = n_threads or os.cpu_count() or 1
        rc = lib().orc_step(self.h, _dp(params_vector(params, guard_c, guard_l)), E, _dp(root), _dp(dof), _dp(act),
                            _dp(pt), _dp(vt), _dp(out["root"]), _dp(out["dof"]), _dp(out["qdd_free"]), r_cap,
                            _ip(out["row_count"]), _ip(out["row_key"]), _dp(out["row_lambda"]),
                            _dp(out["contact_force"]), _dp(out["contact_scale"]), _dp(out["dof_force"]),
                            _ip(out["near"]),
                            out["mode"].ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nt)
        if rc != 0:
            raise ValueError("oracle: bad step arguments")
        return out

    def rollout(self, params, root, dof, actions, pos_targets=None, n_threads=None):
        """FP64 rollout over actions (T, E, D); returns the state before every step."""
        roots, dofs = [root.copy()], [dof.copy()]
        for t in range(actions.shape[0]):
            o = self.step(params, roots[-1], dofs[-1], actions[t],
                          None if pos_targets is None else pos_targets[t], n_threads=n_threads)
            roots.append(o["root"])
            dofs.append(o["dof"])
        return np.stack(roots), np.stack(dofs)
