"""Run one call of step_rk4 on each implementation of the D = 81 stage
(dense MFMA per-stage, structured per-stage, plaquette, 27-row fused) on the
32x32 lattice with 2x2 clusters and d = 3, for profiling them side by side:

    python -m paper_2404_18594_amd.compare_paths [n_traj] [n_steps]
"""
from __future__ import annotations

import os
import sys

import torch

from . import F32, F64, Plan, Problem

PATHS = (("dense", F32), ("generic", F32), ("plaq", F32), ("fused27", F64))


def main(n_traj: int = 32, n_steps: int = 10):
    old = os.environ.get("CDTWA_PATH")
    try:
        for path, dtype in PATHS:
            os.environ["CDTWA_PATH"] = path
            plan = Plan(Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype), n_traj)
            rho = plan.new_state()
            ws = plan.new_workspace()
            plan.sample_noise(5, 0, rho)
            plan.step_rk4(rho, ws, 0.01, n_steps)
            torch.cuda.synchronize()
            print(path, "path", plan.path, "done", flush=True)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


if __name__ == "__main__":
    main(*[int(a) for a in sys.argv[1:3]])
