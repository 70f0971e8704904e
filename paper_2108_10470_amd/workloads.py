"""Seeded synthetic inputs: robot descriptions, initial states and control tensors.

This module only *describes* inputs.  It holds none of the simulation's
arithmetic: no mass properties, no kinematics, no contact geometry.  Both the
FP64 oracle (test infrastructure) and the HIP library read the plain numbers
produced here, each with its own code.

Morphologies follow the workloads the paper benchmarks (Ant with 8 actuated
DOFs and Humanoid with 21, Section 6.1; sim dt 1/120 s and control dt 1/60 s,
Table 4).  The paper ships no asset files, so every dimension below is a
synthetic stand-in with the stated DOF counts.

Random numbers come from a counter-based generator (splitmix64 keyed by seed,
stream and element index) so any slice of a run can be regenerated alone.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

INF = float("inf")

# ----------------------------------------------------------------------------
# counter-based RNG (splitmix64 finaliser, Steele/Lea/Flood 2014)
# ----------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def uniform(seed: int, stream: int, shape, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """U[lo, hi) in float64; element i of the flattened array uses counter i."""
    n = int(np.prod(shape)) if len(shape) else 1
    key = _splitmix64(np.array([(seed & 0xFFFFFFFF) << 32 | (stream & 0xFFFFFFFF)], dtype=np.uint64))[0]
    ctr = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        bits = _splitmix64(ctr ^ key)
    u = (bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (lo + (hi - lo) * u).reshape(shape)


# streams used below (fixed numbering so data stays stable)
STREAM_LIMITS = 1
STREAM_INIT_Q = 2
STREAM_ACTIONS = 3
STREAM_TARGETS = 4
STREAM_PERTURB = 5
STREAM_PROPS = 6


# ----------------------------------------------------------------------------
# description records
# ----------------------------------------------------------------------------
@dataclass
class Shape:
    kind: str                      # 'sphere' | 'capsule' | 'box'
    p0: Tuple[float, float, float]  # sphere/box centre, capsule first cap centre (link frame)
    p1: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # capsule second cap centre
    radius: float = 0.0
    half: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # box half extents (axis aligned in link frame)
    density: float = 1000.0


@dataclass
class Link:
    name: str
    parent: int                    # actor-local index, -1 for the root link
    joint: str                     # root: 'free' | 'fixed'; others: 'revolute' | 'prismatic'
    anchor: Tuple[float, float, float] = (0.0, 0.0, 0.0)  # joint origin in the parent link frame
    axis: Tuple[float, float, float] = (0.0, 0.0, 1.0)    # unit joint axis (parent frame == child frame at q = 0)
    lower: float = -INF
    upper: float = INF
    kp: float = 0.0                # PD drive stiffness
    kd: float = 0.0                # PD drive damping
    armature: float = 0.0
    mass: float = 0.0              # >0: link mass given, shapes only set its distribution
    gear: float = 0.0              # task-level action scale (used by the generator only)
    shapes: List[Shape] = field(default_factory=list)


@dataclass
class Tendon:
    """Fixed tendon (appendix on tendons): a tree of tendon joints, each following the incoming joint of one
    link with a coefficient; the length at a tendon joint is its parent's length plus coefficient x joint
    position.  At every tendon joint a spring (stiffness about rest_length), a damper on the length rate and a
    limit spring (limit_stiffness beyond [lower, upper]) act along the path from the tendon's root."""
    links: List[int]               # per tendon joint: actor-local link (not the root) whose joint it follows
    parents: List[int]             # per tendon joint: parent tendon joint, -1 for the root (parents first)
    coefs: List[float]
    stiffness: float = 0.0
    damping: float = 0.0
    rest_length: float = 0.0
    lower: float = -INF
    upper: float = INF
    limit_stiffness: float = 0.0


@dataclass
class Actor:
    name: str
    links: List[Link]
    root_pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    root_quat: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 1.0)  # xyzw
    init_q_halfwidth: float = 0.0  # joints start at U[-w, w] clipped into limits
    tendons: List[Tendon] = field(default_factory=list)

    @property
    def fixed_base(self) -> bool:
        return self.links[0].joint == "fixed"

    @property
    def dof_links(self) -> List[int]:
        return [i for i, l in enumerate(self.links) if i > 0]

    @property
    def n_dof(self) -> int:
        return len(self.links) - 1


@dataclass
class Pair:
    """Collision pair: shape (actor, link, shape index in link) vs the ground plane (b_actor = -1) or a box."""
    a_actor: int
    a_link: int
    a_shape: int
    b_actor: int = -1
    b_link: int = -1
    b_shape: int = -1


@dataclass
class EnvSpec:
    name: str
    actors: List[Actor]
    pairs: List[Pair]

    @property
    def n_dof(self) -> int:
        return sum(a.n_dof for a in self.actors)

    @property
    def n_actors(self) -> int:
        return len(self.actors)

    @property
    def n_bodies(self) -> int:
        return sum(len(a.links) for a in self.actors)

    @property
    def n_v(self) -> int:
        return sum((0 if a.fixed_base else 6) + a.n_dof for a in self.actors)

    @property
    def n_q(self) -> int:
        return sum((0 if a.fixed_base else 7) + a.n_dof for a in self.actors)


@dataclass
class SimParams:
    dt: float = 1.0 / 60.0
    substeps: int = 2
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    pgs_iters: int = 8
    mu: float = 1.0
    baumgarte: float = 0.2
    contact_margin: float = 0.01
    limit_margin_rev: float = 0.05
    limit_margin_pri: float = 0.005
    solver: int = 0  # 0 projected Gauss-Seidel, 1 its temporal (TGS) variant


# ----------------------------------------------------------------------------
# morphologies
# ----------------------------------------------------------------------------
def _capsule(p0, p1, r, density=1000.0):
    return Shape("capsule", tuple(map(float, p0)), tuple(map(float, p1)), float(r), density=density)


def ant(limit_deg_hip: float = 40.0, limit_deg_knee: float = 70.0, gear: float = 15.0) -> Actor:
    """Ant-like quadruped: torso sphere r=0.25 on a free root, 4 legs of 2 capsule links (r=0.08,
    lengths 0.28 / 0.56), hip axis z and knee axis z x d_k, 8 revolute DOFs."""
    links = [Link("torso", -1, "free", shapes=[Shape("sphere", (0.0, 0.0, 0.0), radius=0.25)])]
    hip = math.radians(limit_deg_hip)
    knee = math.radians(limit_deg_knee)
    for k, deg in enumerate((45.0, 135.0, 225.0, 315.0)):
        th = math.radians(deg)
        d = (math.cos(th), math.sin(th), 0.0)
        thigh_end = (0.28 * d[0], 0.28 * d[1], 0.0)
        # shin direction 0.5*d - (sqrt(3)/2)*z has unit length
        sd = (0.5 * d[0], 0.5 * d[1], -math.sqrt(3.0) / 2.0)
        shin_end = (0.56 * sd[0], 0.56 * sd[1], 0.56 * sd[2])
        links.append(Link(f"hip{k}", 0, "revolute", anchor=(0.25 * d[0], 0.25 * d[1], 0.0),
                          axis=(0.0, 0.0, 1.0), lower=-hip, upper=hip, gear=gear,
                          shapes=[_capsule((0, 0, 0), thigh_end, 0.08)]))
        links.append(Link(f"knee{k}", len(links) - 1, "revolute", anchor=thigh_end,
                          axis=(-d[1], d[0], 0.0), lower=-knee, upper=knee, gear=gear,
                          shapes=[_capsule((0, 0, 0), shin_end, 0.08)]))
    return Actor("ant", links, root_pos=(0.0, 0.0, 0.62), init_q_halfwidth=0.1)


_AXES = {"x": (1.0, 0.0, 0.0), "y": (0.0, 1.0, 0.0), "z": (0.0, 0.0, 1.0)}


def humanoid(limit_seed: int = 0, gear: float = 67.5, armature: float = 0.02, damping: float = 1.0) -> Actor:
    """Humanoid-like: 13 capsule bodies, free root, 21 revolute DOFs.  Multi-axis joints are chains
    of 1-DOF revolutes through massless links whose anchors coincide (the last link of a chain
    carries the capsule).  Joint limits are +-w with w ~ U[0.5, 1.5] seeded per DOF.

    Every DOF has joint armature 0.02 kg m^2 and joint damping 1 N m s/rad (Table 3 lists both as
    per-joint parameters; the values are stand-ins: without them 67.5 N m random torques on ~1 kg
    links make the model itself diverge within a second, even in FP64).

    The torso capsule is centred on the root frame so that the free root frame sits at the root
    centre of mass (the root-state position is the root COM)."""
    # (name, parent name, anchor in parent frame, axes, capsule p0, capsule p1, radius)
    spec = [
        ("abdomen", "torso", (0, 0, -0.27), "zy", (0, 0, 0), (0, 0, -0.10), 0.08),
        ("pelvis", "abdomen", (0, 0, -0.16), "x", (0, -0.07, -0.04), (0, 0.07, -0.04), 0.09),
        ("thigh_r", "pelvis", (0, -0.10, -0.10), "xzy", (0, 0, 0), (0, 0, -0.34), 0.06),
        ("shin_r", "thigh_r", (0, 0, -0.42), "y", (0, 0, 0), (0, 0, -0.30), 0.05),
        ("foot_r", "shin_r", (0, 0, -0.40), "yx", (-0.04, 0, -0.02), (0.12, 0, -0.02), 0.04),
        ("thigh_l", "pelvis", (0, 0.10, -0.10), "xzy", (0, 0, 0), (0, 0, -0.34), 0.06),
        ("shin_l", "thigh_l", (0, 0, -0.42), "y", (0, 0, 0), (0, 0, -0.30), 0.05),
        ("foot_l", "shin_l", (0, 0, -0.40), "yx", (-0.04, 0, -0.02), (0.12, 0, -0.02), 0.04),
        ("uarm_r", "torso", (0, -0.18, 0.09), "xy", (0, 0, 0), (0, 0, -0.24), 0.045),
        ("larm_r", "uarm_r", (0, 0, -0.28), "y", (0, 0, 0), (0, 0, -0.24), 0.04),
        ("uarm_l", "torso", (0, 0.18, 0.09), "xy", (0, 0, 0), (0, 0, -0.24), 0.045),
        ("larm_l", "uarm_l", (0, 0, -0.28), "y", (0, 0, 0), (0, 0, -0.24), 0.04),
    ]
    n_dof = sum(len(s[3]) for s in spec)
    w = uniform(limit_seed, STREAM_LIMITS, (n_dof,), 0.5, 1.5)
    links = [Link("torso", -1, "free", shapes=[_capsule((0, 0, -0.15), (0, 0, 0.15), 0.10)])]
    index = {"torso": 0}
    j = 0
    for name, pname, anchor, axes, c0, c1, r in spec:
        parent = index[pname]
        for ai, ax in enumerate(axes):
            last = ai == len(axes) - 1
            links.append(Link(name if last else f"{name}_{ax}", parent, "revolute",
                              anchor=tuple(map(float, anchor)) if ai == 0 else (0.0, 0.0, 0.0),
                              axis=_AXES[ax], lower=-float(w[j]), upper=float(w[j]), gear=gear,
                              armature=armature, kd=damping, shapes=[_capsule(c0, c1, r)] if last else []))
            j += 1
            parent = len(links) - 1
        index[name] = len(links) - 1
    return Actor("humanoid", links, root_pos=(0.0, 0.0, 1.43), init_q_halfwidth=0.1)


def pendulum(length: float = 0.5, radius: float = 0.05, axis=(0.0, 1.0, 0.0), mass: float = 0.0) -> Actor:
    """Fixed-base single pendulum: one revolute link carrying a capsule hanging along -z."""
    links = [Link("base", -1, "fixed"),
             Link("rod", 0, "revolute", axis=axis, mass=mass,
                  shapes=[_capsule((0, 0, 0), (0, 0, -length), radius)])]
    return Actor("pendulum", links, root_pos=(0.0, 0.0, 2.0))


def double_pendulum(l1=0.5, l2=0.4, r1=0.05, r2=0.04) -> Actor:
    links = [Link("base", -1, "fixed"),
             Link("rod1", 0, "revolute", axis=(0.0, 1.0, 0.0), shapes=[_capsule((0, 0, 0), (0, 0, -l1), r1)]),
             Link("rod2", 1, "revolute", anchor=(0.0, 0.0, -l1), axis=(0.0, 1.0, 0.0),
                  shapes=[_capsule((0, 0, 0), (0, 0, -l2), r2)])]
    return Actor("double_pendulum", links, root_pos=(0.0, 0.0, 3.0))


def free_sphere(radius=0.1, z=0.5) -> Actor:
    return Actor("sphere", [Link("ball", -1, "free", shapes=[Shape("sphere", (0.0, 0.0, 0.0), radius=radius)])],
                 root_pos=(0.0, 0.0, z))


def free_box(half=(0.025, 0.025, 0.025), mass=0.0, pos=(0.0, 0.0, 0.5), density=1000.0) -> Actor:
    return Actor("box", [Link("box", -1, "free", mass=mass,
                              shapes=[Shape("box", (0.0, 0.0, 0.0), half=tuple(half), density=density)])],
                 root_pos=tuple(pos))


def arm_with_gripper(armature: float = 0.1, damping: float = 2.0, finger_armature: float = 0.05,
                     finger_damping: float = 1.0) -> Actor:
    """Fixed-base 7-DOF serial arm (capsules len 0.3, r 0.05, axes z,y,z,y,z,y,z, limits +-2 rad)
    with a 2-finger prismatic gripper (finger capsules len 0.05, r 0.01, range [0, 0.04] m).

    Arm joints carry armature 0.1 kg m^2 and damping 2 N m s/rad, fingers 0.05 kg and 1 N s/m (Table 3
    joint parameters; stand-in values): the z-axis joints turn a capsule about its own axis
    (~0.005 kg m^2), and without them +-20 N m random torques slam them between their limits at
    ~70 rad/s every step, a state in which a rounding-level perturbation grows without bound."""
    links = [Link("base", -1, "fixed")]
    for k, ax in enumerate("zyzyzyz"):
        links.append(Link(f"link{k}", len(links) - 1, "revolute",
                          anchor=(0.0, 0.0, 0.1 if k == 0 else 0.3), axis=_AXES[ax],
                          lower=-2.0, upper=2.0, gear=20.0, armature=armature, kd=damping,
                          shapes=[_capsule((0, 0, 0), (0, 0, 0.3), 0.05)]))
    hand = len(links) - 1
    for side in (1.0, -1.0):
        links.append(Link(f"finger{'l' if side > 0 else 'r'}", hand, "prismatic",
                          anchor=(0.0, 0.0, 0.36), axis=(0.0, side, 0.0), lower=0.0, upper=0.04, gear=10.0,
                          armature=finger_armature, kd=finger_damping,
                          shapes=[_capsule((0, 0, 0), (0, 0, 0.05), 0.01)]))
    return Actor("arm", links, root_pos=(0.0, 0.0, 0.0), init_q_halfwidth=0.1)


def hand(kp: float = 3.0, kd: float = 0.1, z: float = 0.3) -> Actor:
    """Fixed-base hand-like tree with 24 DOFs, palm up: palm box 0.10 x 0.10 x 0.02 m carrying three palm-top
    capsules (r 0.01) so that palm-object contact is capsule-box, four fingers of five links (abduction about
    the palm normal, then four flexions) along +x and a four-link thumb along -y.  Finger capsules have
    r = 0.01 and lengths 0.05, 0.04, 0.04, 0.03, 0.03; flexion limits [0, 1.57], abduction +-0.35.
    Every DOF is driven by a PD drive (kp, kd)."""
    palm_shapes = [Shape("box", (0.0, 0.0, 0.0), half=(0.05, 0.05, 0.01))]
    for x in (-0.03, 0.0, 0.03):
        palm_shapes.append(_capsule((x, -0.04, 0.0), (x, 0.04, 0.0), 0.01))
    links = [Link("palm", -1, "fixed", shapes=palm_shapes)]
    lengths = (0.05, 0.04, 0.04, 0.03, 0.03)

    def chain(name, base_anchor, along, flex_axis, n_links):
        parent = 0
        anchor = base_anchor
        for k in range(n_links):
            L = lengths[k]
            tip = tuple(L * a for a in along)
            if k == 0:
                links.append(Link(f"{name}_abd", parent, "revolute", anchor=anchor, axis=(0.0, 0.0, 1.0),
                                  lower=-0.35, upper=0.35, kp=kp, kd=kd, gear=1.0, shapes=[_capsule((0, 0, 0), tip, 0.01)]))
            else:
                links.append(Link(f"{name}_f{k}", parent, "revolute", anchor=anchor, axis=flex_axis,
                                  lower=0.0, upper=1.57, kp=kp, kd=kd, gear=1.0, shapes=[_capsule((0, 0, 0), tip, 0.01)]))
            parent = len(links) - 1
            anchor = tip

    for i, y in enumerate((-0.0375, -0.0125, 0.0125, 0.0375)):
        chain(f"finger{i}", (0.06, y, 0.0), (1.0, 0.0, 0.0), (0.0, -1.0, 0.0), 5)
    chain("thumb", (-0.02, -0.06, 0.0), (0.0, -1.0, 0.0), (-1.0, 0.0, 0.0), 4)
    return Actor("hand", links, root_pos=(0.0, 0.0, z))


# ----------------------------------------------------------------------------
# environments (actors + collision pairs)
# ----------------------------------------------------------------------------
def _plane_pairs(actors: Sequence[Actor]) -> List[Pair]:
    pairs = []
    for ai, a in enumerate(actors):
        for li, l in enumerate(a.links):
            for si, _ in enumerate(l.shapes):
                pairs.append(Pair(ai, li, si))
    return pairs


def env_single(actor: Actor, ground: bool = True) -> EnvSpec:
    return EnvSpec(actor.name, [actor], _plane_pairs([actor]) if ground else [])


def env_ant() -> EnvSpec:
    return env_single(ant())


def env_humanoid(limit_seed: int = 0) -> EnvSpec:
    return env_single(humanoid(limit_seed))


def env_arm_box() -> EnvSpec:
    arm = arm_with_gripper()
    box = free_box(half=(0.025, 0.025, 0.025), mass=0.125, pos=(0.4, 0.0, 0.025))
    actors = [arm, box]
    pairs = _plane_pairs(actors)
    for li, l in enumerate(arm.links):
        for si, s in enumerate(l.shapes):
            if s.kind == "capsule":
                pairs.append(Pair(0, li, si, 1, 0, 0))
    return EnvSpec("arm_box", actors, pairs)


def add_finger_tendons(h: Actor, stiffness: float = 0.3, damping: float = 0.01, lower: float = -0.4,
                       upper: float = 1.6, limit_stiffness: float = 3.0) -> Actor:
    """One fixed tendon per finger of the hand coupling its last two flexions (as the hand of the paper's
    Shadow Hand experiments couples a finger's distal joints): root tendon joint on the third flexion
    (coefficient 1), child on the fourth (coefficient -1), rest length 0, so the child's length is the
    difference of the two flexions.  The forces are explicit (start-of-substep state): the stiffnesses are
    chosen so that (k + limit k) h^2 stays well below the joints' effective inertia (about 1e-3 kg m^2, most
    of it the implicit drive's h kd + h^2 kp)."""
    names = [l.name for l in h.links]
    for i in range(4):
        a, b = names.index(f"finger{i}_f3"), names.index(f"finger{i}_f4")
        h.tendons.append(Tendon([a, b], [-1, 0], [1.0, -1.0], stiffness=stiffness, damping=damping,
                                lower=lower, upper=upper, limit_stiffness=limit_stiffness))
    return h


def env_hand_cube(z: float = 0.3, tendons: bool = False) -> EnvSpec:
    """The hand holding a free cube (edge 0.065 m, 0.1 kg) that rests on the palm-top capsules; pairs: every
    capsule of the hand against the cube, and the cube against the ground.  tendons: add the finger
    tendons (add_finger_tendons)."""
    h = hand(z=z)
    if tendons:
        add_finger_tendons(h)
    cube = free_box(half=(0.0325, 0.0325, 0.0325), mass=0.1, pos=(0.0, 0.0, z + 0.01 + 0.0325))
    actors = [h, cube]
    pairs = []
    for li, l in enumerate(h.links):
        for si, sh in enumerate(l.shapes):
            if sh.kind == "capsule":
                pairs.append(Pair(0, li, si, 1, 0, 0))
    pairs.append(Pair(1, 0, 0))
    return EnvSpec("hand_cube", actors, pairs)


HAND_PARAMS = SimParams(pgs_iters=12, contact_margin=0.003)


# ----------------------------------------------------------------------------
# seeded state and control tensors (paper Tables 1-2 layouts)
# ----------------------------------------------------------------------------
def initial_state(env: EnvSpec, n_envs: int, seed: int = 0):
    """Actor root states (n_envs, n_actors, 13) = pos, quat xyzw, linvel, angvel, and
    DOF states (n_envs, n_dof, 2) = position, velocity; float64."""
    root = np.zeros((n_envs, env.n_actors, 13))
    for ai, a in enumerate(env.actors):
        root[:, ai, 0:3] = a.root_pos
        root[:, ai, 3:7] = a.root_quat
    dof = np.zeros((n_envs, env.n_dof, 2))
    u = uniform(seed, STREAM_INIT_Q, (n_envs, env.n_dof), -1.0, 1.0)
    j = 0
    for a in env.actors:
        for li in a.dof_links:
            l = a.links[li]
            q = a.init_q_halfwidth * u[:, j]
            dof[:, j, 0] = np.clip(q, l.lower, l.upper)
            j += 1
    return root, dof


def gears(env: EnvSpec) -> np.ndarray:
    return np.array([a.links[li].gear for a in env.actors for li in a.dof_links], dtype=np.float64)


def actuation(env: EnvSpec, n_envs: int, n_steps: int, seed: int = 0, step0: int = 0) -> np.ndarray:
    """DOF actuation forces (n_steps, n_envs, n_dof): U[-1, 1] x gear per DOF."""
    g = gears(env)
    total = uniform(seed, STREAM_ACTIONS, (step0 + n_steps, n_envs, env.n_dof), -1.0, 1.0)[step0:]
    return total * g[None, None, :]


def pd_targets(env: EnvSpec, n_envs: int, n_steps: int, seed: int = 0) -> np.ndarray:
    """DOF position targets (n_steps, n_envs, n_dof) drawn uniformly inside each DOF's limits."""
    lo = np.array([a.links[li].lower for a in env.actors for li in a.dof_links])
    hi = np.array([a.links[li].upper for a in env.actors for li in a.dof_links])
    u = uniform(seed, STREAM_TARGETS, (n_steps, n_envs, env.n_dof))
    return lo + (hi - lo) * u


PARAMS_DEFAULT = SimParams()


# ----------------------------------------------------------------------------
# single-precision-representable copies (the library's description structs are float32)
# ----------------------------------------------------------------------------
def _r32(x):
    return float(np.float32(x))


def as_f32(env: EnvSpec) -> EnvSpec:
    """Deep copy of env with every number rounded to float32, so that a consumer reading float32
    fields and one reading float64 fields see identical values."""
    import copy
    e = copy.deepcopy(env)
    for a in e.actors:
        a.root_pos = tuple(_r32(v) for v in a.root_pos)
        a.root_quat = tuple(_r32(v) for v in a.root_quat)
        for l in a.links:
            l.anchor = tuple(_r32(v) for v in l.anchor)
            l.axis = tuple(_r32(v) for v in l.axis)
            for f in ("lower", "upper", "kp", "kd", "armature", "mass", "gear"):
                setattr(l, f, _r32(getattr(l, f)))
            for sh in l.shapes:
                sh.p0 = tuple(_r32(v) for v in sh.p0)
                sh.p1 = tuple(_r32(v) for v in sh.p1)
                sh.half = tuple(_r32(v) for v in sh.half)
                sh.radius = _r32(sh.radius)
                sh.density = _r32(sh.density)
        for t in a.tendons:
            t.coefs = [_r32(c) for c in t.coefs]
            for f in ("stiffness", "damping", "rest_length", "lower", "upper", "limit_stiffness"):
                setattr(t, f, _r32(getattr(t, f)))
    return e


def _normal(seed: int, stream: int, shape) -> np.ndarray:
    """Standard normals by Box-Muller from two uniform streams."""
    u1 = uniform(seed, stream, shape, 0.0, 1.0)
    u2 = uniform(seed, stream + 1000, shape, 0.0, 1.0)
    return np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)


def random_properties(env: EnvSpec, params: SimParams, n_envs: int, seed: int = 0) -> dict:
    """Per-env physical properties drawn as in the paper's table of physics randomizations (hand
    experiments): link masses x U[0.5, 1.5], friction x U[0.7, 1.3], joint damping x loguniform[0.3, 3],
    drive stiffness (P gain) x loguniform[0.75, 1.5], joint limits + N(0, 0.15) (radians; prismatic limits
    scaled to metres by 0.1), gravity + N(0, 0.4) per coordinate.  Float32 arrays shaped like the sim's
    property tensors: mass_scale (E, N_B/E), stiffness, damping (E, D), limits (E, D, 2), friction (E,),
    gravity (E, 3).  Limits stay ordered (lower <= upper)."""
    nb, nd = env.n_bodies, env.n_dof
    base = seed * 16 + 7
    links = [l for a in env.actors for l in a.links[1:]]
    kp = np.array([l.kp for l in links])
    kd = np.array([l.kd for l in links])
    lo = np.array([l.lower for l in links])
    hi = np.array([l.upper for l in links])
    scale_lim = np.array([0.1 if l.joint == "prismatic" else 1.0 for l in links])
    lu = lambda k, a, b: np.exp(uniform(base, STREAM_PROPS * 100 + k, (n_envs, nd), np.log(a), np.log(b)))
    dlo = 0.15 * scale_lim * _normal(base, STREAM_PROPS * 100 + 3, (n_envs, nd))
    dhi = 0.15 * scale_lim * _normal(base, STREAM_PROPS * 100 + 4, (n_envs, nd))
    nlo, nhi = lo + dlo, hi + dhi
    swap = nlo > nhi
    nlo[swap], nhi[swap] = (nlo[swap] + nhi[swap]) / 2, (nlo[swap] + nhi[swap]) / 2
    out = {
        "mass_scale": uniform(base, STREAM_PROPS * 100 + 0, (n_envs, nb), 0.5, 1.5),
        "stiffness": kp * lu(1, 0.75, 1.5),
        "damping": kd * lu(2, 0.3, 3.0),
        "limits": np.stack([nlo, nhi], axis=-1),
        "friction": params.mu * uniform(base, STREAM_PROPS * 100 + 5, (n_envs,), 0.7, 1.3),
        "gravity": np.array(params.gravity) + 0.4 * _normal(base, STREAM_PROPS * 100 + 6, (n_envs, 3)),
    }
    return {k: v.astype(np.float32) for k, v in out.items()}


def env_with_properties(env: EnvSpec, params: SimParams, props: dict, e: int):
    """The model and parameters that env e of a batch with per-env properties `props` (as returned by
    random_properties, float32) simulates: link masses and inertias scaled by scaling every shape's density
    (and a given mass), drive gains and limits replaced, friction and gravity in the parameters."""
    import copy
    import dataclasses
    spec = copy.deepcopy(env)
    b = d = 0
    for a in spec.actors:
        for i, l in enumerate(a.links):
            s = float(props["mass_scale"][e, b])
            if l.mass > 0:
                l.mass = l.mass * s
            for sh in l.shapes:
                sh.density = sh.density * s
            if i > 0:
                l.kp = float(props["stiffness"][e, d])
                l.kd = float(props["damping"][e, d])
                l.lower = float(props["limits"][e, d, 0])
                l.upper = float(props["limits"][e, d, 1])
                d += 1
            b += 1
    p = dataclasses.replace(params, mu=float(props["friction"][e]), gravity=tuple(float(g) for g in props["gravity"][e]))
    return spec, p


def params_f32(p: SimParams) -> SimParams:
    """Copy of p with every float parameter rounded to float32."""
    return SimParams(dt=_r32(p.dt), substeps=p.substeps, gravity=tuple(_r32(g) for g in p.gravity),
                     pgs_iters=p.pgs_iters, mu=_r32(p.mu), baumgarte=_r32(p.baumgarte),
                     contact_margin=_r32(p.contact_margin), limit_margin_rev=_r32(p.limit_margin_rev),
                     limit_margin_pri=_r32(p.limit_margin_pri), solver=p.solver)
