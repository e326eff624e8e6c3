"""Writes oracle_c1_regression.json: states of the FP64 oracle on the 64-env
BlueROV2 workload (seeded inputs, dt = 0.01 s, linear thrust map, no lag) at a
few control steps.  It calls only the oracle and the seeded input generators;
the fixture guards the oracle against unintended changes (its physics is
pinned by the closed-form tests, not by this file).

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from workloads import BLUEROV2, CONFIGS, initial_state, actions  # noqa: E402

STEPS = [1, 10, 100, 1000]
ENVS = [0, 17, 63]


def main():
    c = CONFIGS["c1"]
    x0 = initial_state(c.n_envs, 13, c.seed_base + 2)
    act = actions(c.n_ctrl, 6, c.n_envs, c.seed_base + 3)
    out = O.rollout(BLUEROV2, x0, act, c.substeps, c.dt_sub, want_traj=True, want_stats=True)
    fixture = {
        "what": "FP64 oracle, 64 BlueROV2 envs, seeds 1002/1003, dt 0.01, linear map, no lag",
        "steps": STEPS, "envs": ENVS,
        "states": {str(t): {str(e): out["traj"][t - 1, :, e].tolist() for e in ENVS} for t in STEPS},
        "stats": {str(t): out["stats"][t - 1].tolist() for t in STEPS},
    }
    with open(os.path.join(HERE, "oracle_c1_regression.json"), "w") as f:
        json.dump(fixture, f, indent=1)


if __name__ == "__main__":
    main()
