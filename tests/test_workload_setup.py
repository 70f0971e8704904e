"""The synthetic workloads against the simulation setup the paper prints for its environments
(tests/golden/sim_setup_table.txt: the table "Simulation setup for the environments", section Environments).
CPU only."""
import os
from fractions import Fraction

import pytest

from paper_2108_10470_amd import ags, workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sim_setup_table.txt")


def _table():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, sim_dt, ctrl_dt, dims = (x.strip() for x in line.split("|"))
            rows[name] = (Fraction(sim_dt), Fraction(ctrl_dt), int(dims))
    return rows


# workload model and its parameters for each row; action dims compared where the stand-in drives the same
# number of DOFs (the hand-like stand-in drives all 24 joints, the paper's hand 20 of them)
CASES = {"Ant": (W.env_ant, W.SimParams(), True), "Humanoid": (W.env_humanoid, W.SimParams(), True),
         "Shadow Hand Standard": (W.env_hand_cube, W.HAND_PARAMS, False)}


@pytest.mark.parametrize("name", sorted(CASES))
def test_workload_matches_the_papers_simulation_setup(name):
    sim_dt, ctrl_dt, dims = _table()[name]
    env_fn, params, same_dims = CASES[name]
    # one control step per env-step (the actions are held over its substeps)
    assert Fraction(params.dt).limit_denominator(1000) == ctrl_dt
    assert Fraction(params.dt / params.substeps).limit_denominator(1000) == sim_dt
    if same_dims:
        env = env_fn()
        assert env.n_dof == dims
        assert ags.Model(env).info.n_dof == dims
