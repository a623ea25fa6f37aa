"""Quench driver: sample -> RK4 -> observables through the C ABI, batched
over trajectories so that the state and the RK4 workspace fit in HBM."""
from __future__ import annotations

import torch

from .binding import NOBS, Plan, Problem


def run_quench(problem: Problem, n_traj: int, seed: int, dt: float, record_steps, traj_offset: int = 0,
               batch: int | None = None, want_per_traj: bool = True, stream=None):
    """The initial state of `problem` (Mott state, or the Ising start) quenched
    to its couplings.

    Returns (sums [n_rec][NOBS][3] float64 on the host, per_traj
    [n_traj][n_rec][NOBS] float64 on the host or None).  `record_steps` are
    ascending step counts (0 = initial state)."""
    rec = [int(s) for s in record_steps]
    if any(b <= a for a, b in zip(rec, rec[1:])) or (rec and rec[0] < 0):
        raise ValueError("record_steps must be ascending and non-negative")
    batch = int(batch or n_traj)
    sums = torch.zeros(len(rec), NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(n_traj, len(rec), NOBS, dtype=torch.float64) if want_per_traj else None
    plan = None
    done = 0
    while done < n_traj:
        nb = min(batch, n_traj - done)
        if plan is None or plan.n_traj != nb:
            plan = Plan(problem, nb)
            rho = plan.new_state()
            ws = plan.new_workspace()
            ptr = torch.empty(len(rec), nb, NOBS, dtype=torch.float64, device="cuda")
        plan.sample_noise(seed, traj_offset + done, rho, stream=stream)
        step = 0
        for k, s in enumerate(rec):
            if s > step:
                plan.step_rk4(rho, ws, dt, s - step, stream=stream)
                step = s
            plan.accumulate_observables(rho, k, sums, ws, per_traj=ptr[k], stream=stream)
        if per is not None:
            per[done:done + nb] = ptr.transpose(0, 1).cpu()
        done += nb
    torch.cuda.synchronize()
    return sums.cpu(), per


def estimates(sums: torch.Tensor, n: int):
    """Mean and standard error from the compensated sums."""
    s = sums[..., 0] + sums[..., 1]
    mean = s / n
    var = (sums[..., 2] / n - mean ** 2).clamp_min(0) * n / max(n - 1, 1)
    return mean, (var / n).sqrt()
