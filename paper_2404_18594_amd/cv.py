"""Learned control variate for the C-dTWA estimate of the nearest-neighbour
correlation O = (C^sp_(1,0) + C^sp_(0,1)) / 2 (Sec. III definition of C^sp).

This is an addition to the paper's method, not part of it (the paper uses
plain trajectory averages, Sec. II).  A network g maps the noise of the 4x4
patch around each 2x2 cluster to the cluster's share t_mu of O at up to 64
recorded times; per trajectory G = (1/Ns) sum_mu g(patch_mu).  Because the
site noise is i.i.d., every patch has the law of an i.i.d. patch, so

    mean_traj(O - G) + (n_clusters / Ns) E[g]

is unbiased for any fixed g, with E[g] estimated on fresh i.i.d. patches.
Training, inference, the patch sampler and every reduction run in the HIP
library; this module orders the calls and forms the final statistics.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .binding import MLP_IN, MLP_OUT, NOBS, Mlp, Plan, Problem, new_cv_workspace


def record_schedule(n_steps: int, n_times: int = MLP_OUT):
    """Up to n_times distinct steps spread evenly over 0..n_steps."""
    return sorted({int(round(k * n_steps / (n_times - 1))) for k in range(n_times)})


@dataclass
class Simulation:
    features: torch.Tensor      # [n_traj * nc][128] float32
    targets: torch.Tensor       # [n_traj * nc][64] float32 (columns past the schedule are 0) or None
    per_traj: torch.Tensor      # [n_rec][n_traj][NOBS] float64 or None
    plan: Plan


def simulate(problem: Problem, n_traj: int, seed: int, traj_offset: int, dt: float, record_steps,
             want_obs: bool = True, want_targets: bool = True, stream=None) -> Simulation:
    """Sample, integrate and record features, per-cluster targets (when
    want_targets) and per-trajectory observables (when want_obs) at every
    recorded step."""
    rec = [int(s) for s in record_steps]
    if len(rec) > MLP_OUT:
        raise ValueError(f"at most {MLP_OUT} recorded times")
    plan = Plan(problem, n_traj)
    rho = plan.new_state()
    ws = plan.new_workspace()
    noise = torch.empty(n_traj, plan.n_sites, plan.n_gen, dtype=torch.int8, device="cuda")
    plan.sample_noise(seed, traj_offset, rho, noise=noise, stream=stream)
    feats = torch.empty(n_traj * plan.n_clusters, MLP_IN, dtype=torch.float32, device="cuda")
    plan.cv_features(noise, feats, stream=stream)
    del noise
    targets = torch.zeros(n_traj * plan.n_clusters, MLP_OUT, dtype=torch.float32, device="cuda") \
        if want_targets else None
    per = torch.empty(len(rec), n_traj, NOBS, dtype=torch.float64, device="cuda") if want_obs else None
    sums = torch.zeros(len(rec), NOBS, 3, dtype=torch.float64, device="cuda")
    step = 0
    for k, s in enumerate(rec):
        if s > step:
            plan.step_rk4(rho, ws, dt, s - step, stream=stream)
            step = s
        if want_targets:
            plan.cv_targets(rho, k, targets, ws, stream=stream)
        if want_obs:
            plan.accumulate_observables(rho, k, sums, ws, per_traj=per[k], stream=stream)
    return Simulation(feats, targets, per, plan)


def train(mlp: Mlp, features: torch.Tensor, targets: torch.Tensor, epochs: int, batch: int = 4096,
          lr: float = 1e-3, stream=None):
    """Adam on the mean squared error over contiguous minibatches (rows of
    consecutive trajectories; trajectories are independent).  Returns the
    loss of the last minibatch of every epoch."""
    n = features.shape[0]
    batch = min(batch, n - n % 16)
    if batch < 16:
        raise ValueError("need at least 16 training rows")
    ws = Mlp.new_workspace(batch)
    y = torch.empty(batch, MLP_OUT, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    hist = []
    for _ in range(epochs):
        for b0 in range(0, n - batch + 1, batch):
            mlp.forward(features[b0:b0 + batch], y, ws, stream=stream)
            mlp.backward(y, targets[b0:b0 + batch], ws, loss=loss, stream=stream)
            mlp.adam(lr, stream=stream)
        hist.append(float(loss.item()))
    return hist


def predict(mlp: Mlp, features: torch.Tensor, chunk: int = 65536, stream=None) -> torch.Tensor:
    n = features.shape[0]
    y = torch.empty(n, MLP_OUT, dtype=torch.float32, device="cuda")
    ws = Mlp.new_workspace(min(chunk, n))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        mlp.forward(features[c0:c1], y[c0:c1], ws, stream=stream)
    return y


def expectation(plan: Plan, mlp: Mlp, seed: int, n_samples: int, stream=None):
    """Mean and variance of g over n_samples i.i.d. patches (per output)."""
    mom = torch.zeros(MLP_OUT, 3, dtype=torch.float64, device="cuda")
    plan.cv_expectation(mlp, seed, n_samples, mom, ws=new_cv_workspace(), stream=stream)
    m = mom.cpu().numpy()
    mean = (m[:, 0] + m[:, 1]) / n_samples
    var = np.maximum(m[:, 2] / n_samples - mean ** 2, 0.0) * n_samples / max(n_samples - 1, 1)
    return mean, var


def observable_and_cv(sim: Simulation, mlp: Mlp, stream=None):
    """Per-trajectory O (rows: trajectories, columns: recorded times) and
    G = (1/Ns) sum_mu g(patch_mu) at the same times, as host arrays."""
    plan = sim.plan
    y = predict(mlp, sim.features, stream=stream)
    gtraj = torch.empty(plan.n_traj, MLP_OUT, dtype=torch.float64, device="cuda")
    plan.cv_traj_sums(y, gtraj, stream=stream)
    per = sim.per_traj.cpu().numpy()                  # [n_rec][n][NOBS]
    n_rec = per.shape[0]
    O = 0.5 * (per[:, :, 0] + per[:, :, 1]).T         # [n][n_rec]
    G = gtraj.cpu().numpy()[:, :n_rec]
    return O, G


def estimate(O: np.ndarray, G: np.ndarray, eg: np.ndarray, varg: np.ndarray, eg_samples: int, c: float):
    """Plain and control-variate estimates of O at every recorded time from
    per-trajectory O and G; c = n_clusters / Ns scales E[g] to E[G].

    Returns a dict of arrays over the recorded times: plain mean and standard
    error, CV mean and standard error (trajectory part and the E[g] part
    combined), and the variance ratio Var(O - G) / Var(O)."""
    n, n_rec = O.shape
    diff = O - G
    plain_var = O.var(axis=0, ddof=1)
    cv_var = diff.var(axis=0, ddof=1)
    return {
        "plain_mean": O.mean(axis=0),
        "plain_se": np.sqrt(plain_var / n),
        "cv_mean": diff.mean(axis=0) + c * eg[:n_rec],
        "cv_se": np.sqrt(cv_var / n + c * c * varg[:n_rec] / eg_samples),
        "var_ratio": cv_var / np.maximum(plain_var, 1e-300),
        "plain_var": plain_var,
        "cv_var": cv_var,
    }
