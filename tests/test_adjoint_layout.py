"""Host-side checks of the adjoint kernel's LDS use (CPU only).

1. tests/adj_lds_check.cpp replays make_adj_layout (the header the runtime uses) for every workload model
   and a grid of substeps, Gauss-Seidel sweeps, row capacities and with or without the staged model tables, touching every index the kernel's
   indexing can reach in buffers of exactly the layout's size, built with AddressSanitizer and UBSan.
2. The adjoint kernels of this build reach LDS only through DS instructions: no FLAT memory instruction
   and no call appears in their gfx950 assembly (long branches within a kernel are allowed).  (An earlier instrumented build, in which the compiler
   outlined the reverse substep into a real call and reached LDS through FLAT instructions with offsets
   beyond 64 KiB, faulted with a memory-aperture violation; the FP64 layouts put their row and tape arrays
   above 64 KiB, as the replay reports.)
"""
import json
import os
import re
import subprocess

import pytest

from paper_2108_10470_amd import ags, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_10470_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("adjlds") / "adj_lds_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", CSRC, "-I", os.path.join(ROOT, "include"), "-o", exe,
                           os.path.join(ROOT, "tests", "adj_lds_check.cpp")])
    return exe


MODELS = {"humanoid": W.env_humanoid, "ant": W.env_ant, "arm_box": W.env_arm_box, "hand_cube": W.env_hand_cube,
          "pendulum": lambda: W.EnvSpec("pend", [W.pendulum()], [])}


@pytest.mark.parametrize("model", sorted(MODELS))
def test_adjoint_lds_layout_replay(checker, model):
    info = ags.Model(MODELS[model]()).info
    out = []
    for substeps in (1, 2, 3):
        for iters in (1, 8, 12, 32):
            for cap, staged in ((5, 0), (32, 0), (32, 1), (64, 1)):
                args = [str(x) for x in (info.n_links, info.n_v, info.n_dof, info.n_actors, info.max_rows, substeps,
                                         iters, cap, staged)]
                r = subprocess.run([checker, *args], capture_output=True, text=True)
                assert r.returncode == 0, (args, r.stderr)
                d = json.loads(r.stdout)
                assert d["ok"], (args, d)
                out.append(d)
    print(model, out[-1])


def test_humanoid_fp64_full_layout_reaches_beyond_64_kib(checker):
    """The configuration of the earlier fault: the FP64 full (64-row) layout of the humanoid-like model puts
    its Delassus, row and tape arrays above 64 KiB of LDS."""
    info = ags.Model(W.env_humanoid()).info
    r = subprocess.run([checker, *[str(x) for x in (info.n_links, info.n_v, info.n_dof, info.n_actors, info.max_rows,
                                                    2, 8, 64, 1)]], capture_output=True, text=True, check=True)
    d = json.loads(r.stdout)
    above = d["above_64KiB_f64"]
    assert d["bytes_f64"] > 65536 and all(x in above for x in ("hst", "Ab", "rbc", "hlo")), d


def test_humanoid_small_layouts_fit_six_fp32_or_three_fp64_workgroups_per_cu(checker):
    """The pass-1 (32-row) layouts of the humanoid-like model, as the runtime builds them (FP32 without and FP64
    with the staged model tables; two substeps, eight sweeps), plus the kernels' 104 B of static LDS, fit six
    (FP32) or three (FP64) workgroups in a CU's 163,840 B of LDS: the reverse pass's throughput rests on it."""
    info = ags.Model(W.env_humanoid()).info
    static_lds, cu_lds = 104, 163840
    sizes = {}
    for staged, key, per_cu in ((0, "bytes_f32", 6), (1, "bytes_f64", 3)):
        r = subprocess.run([checker, *[str(x) for x in (info.n_links, info.n_v, info.n_dof, info.n_actors,
                                                        info.max_rows, 2, 8, 32, staged)]],
                           capture_output=True, text=True, check=True)
        d = json.loads(r.stdout)
        sizes[key] = d[key]
        assert per_cu * (d[key] + static_lds) <= cu_lds, (key, d[key])
    print(sizes)


def test_adjoint_kernels_reach_lds_through_ds_instructions_only(tmp_path):
    asm = tmp_path / "adj.s"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "--cuda-device-only", "-S", "-O3",
                           "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), os.path.join(CSRC, "ags_adjoint.hip"), "-o", str(asm)],
                          stderr=subprocess.DEVNULL)
    text = asm.read_text()
    kernels = re.findall(r"^(_ZN3ags\w*adjoint\w*kernel\w*):", text, flags=re.M)
    assert len(kernels) >= 4, kernels
    for k in kernels:
        body = text.split(f"\n{k}:", 1)[1].split("s_endpgm", 1)[0]
        assert not re.search(r"\bflat_(load|store|atomic)", body), k
        # no call; an s_setpc may only end a long branch to a label of the kernel (s_getpc, then the label's
        # offset added), which the assembler emits when a kernel outgrows the short branch range
        assert "s_swappc" not in body and "s_call" not in body, k
        lines = body.splitlines()
        for n, line in enumerate(lines):
            if "s_setpc_b64" in line:
                window = "\n".join(lines[max(0, n - 4):n])
                assert "s_getpc_b64" in window and re.search(r"\(\.LBB\w+-\.Lpost_getpc\w*\)", window), (k, n)
        assert re.search(r"\bds_(read|write|load|store)", body), k
