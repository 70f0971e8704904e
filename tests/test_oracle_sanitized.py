"""The FP64 oracle built with AddressSanitizer and UBSan (CPU only).

The oracle's C++ is compiled with -fsanitize=address,undefined (no recovery) into a temporary library and
driven through its own ctypes wrapper in a child process that preloads the ASan runtime: every entry point
(mass properties, kinematics, body states, Jacobian, mass matrix, unconstrained dynamics, contact slots,
the step with its rows, limits, tendons and PD targets, and a short rollout) runs on every workload model.
Any out-of-bounds access, use of freed memory or undefined behaviour aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import sys
sys.path.insert(0, ROOT)
import numpy as np
from oracle import oracle as O
O.LIB_PATH = LIB
from paper_2108_10470_amd import workloads as W

models = {"humanoid": W.env_humanoid, "ant": W.env_ant, "arm_box": W.env_arm_box, "hand_cube": W.env_hand_cube,
          "hand_cube_tendons": lambda: W.env_hand_cube(tendons=True)}
for name, make in models.items():
    env = W.as_f32(make())
    p = W.params_f32(W.SimParams())
    oe = O.OracleEnv(env)
    E = 3
    root, dof = W.initial_state(env, E, 1)
    acts = W.actuation(env, E, 4, 1)
    oe.mass_props()
    r1, d1 = root[0], dof[0]  # the single-env entry points
    oe.fk(r1, d1)
    oe.body_states(r1, d1)
    oe.jacobian(r1, d1)
    oe.mass_matrix(r1, d1)
    oe.slots(r1, d1)
    oe.dynamics(p, r1, d1, np.zeros(oe.n_v))
    tgt = W.pd_targets(env, E, 1, 1)[0] if env.n_dof else None
    for t in range(3):
        o = oe.step(p, root, dof, acts[t], pos_tgt=tgt)
        root, dof = o["root"], o["dof"]
    r = oe.rollout(p, root, dof, acts[:2])
    assert np.isfinite(root).all(), name
    print(name, "ok", flush=True)
'''


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-shared", "-fPIC", "-pthread", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", lib,
                           os.path.join(ROOT, "oracle", "oracle.cpp")])
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("no ASan runtime for the host compiler")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + DRIVER
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.count(" ok") == 5, r.stdout
