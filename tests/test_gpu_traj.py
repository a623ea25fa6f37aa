"""Trajectory-resident path (plan path 6): d = 3 with 1x1, 2x1 and 1x2
clusters, whole trajectories on chip for a call, a persistent grid pulling
blocks of trajectories from a work queue.  Every case is compared with the
FP64 oracle on the same noise, entry by entry (Sec. II Eq. (cluster_mf);
App. B.1), over trajectory counts that leave a ragged last block, periodic
and open lattices, and lattices at the sizes of the batching workload."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


def _plan(prob, n, path=None):
    old = os.environ.get("CDTWA_PATH")
    try:
        if path:
            os.environ["CDTWA_PATH"] = path
        else:
            os.environ.pop("CDTWA_PATH", None)
        return cd.Plan(prob, n)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


def _tol(dtype):
    return 1e-12 if dtype == cd.F64 else 2e-5


# (Lx, Ly, cx, cy, periodic, U, blocks): n_traj = blocks * per-workgroup + 1
CASES = [
    (4, 4, 1, 1, True, 5.0, 2),
    (6, 4, 1, 1, False, 3.0, 1),
    (4, 4, 2, 1, True, 10.0, 2),
    (6, 6, 2, 1, False, 5.0, 1),
    (4, 4, 1, 2, True, 3.0, 1),
    (4, 6, 1, 2, False, 5.0, 2),
    (3, 4, 1, 2, True, 5.0, 1),
]


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
@pytest.mark.parametrize("case", CASES)
def test_traj_path_matches_oracle(case, dtype):
    Lx, Ly, cx, cy, periodic, U, blocks = case
    prob = cd.Problem(Lx, Ly, cx, cy, d=3, periodic=periodic, J=1.0, U=U, dtype=dtype)
    probe = _plan(prob, 1)
    assert probe.path == 6, probe.path
    # trajectories per workgroup at this size, then a count with a ragged last block
    big = _plan(prob, 4096)
    n = blocks * big.resident + 1
    plan = _plan(prob, n)
    assert plan.path == 6
    _say("traj", case, "dtype", dtype, "per workgroup", plan.resident, "n_traj", n)
    op = oracle.Problem(Lx, Ly, cx, cy, d=3, periodic=periodic, J=1.0, U=U)
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(500 + blocks, 3, rho)
    plan.step_rk4(rho, ws, 0.01, 5)
    plan.step_rk4(rho, ws, 0.02, 4)
    torch.cuda.synchronize()
    _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=500 + blocks, traj_offset=3, n_traj=n)
    ref = oracle.rk4(op, oracle.rk4(op, r0, 0.01, 5), 0.02, 4)
    got = rho.cpu().numpy().astype(np.complex128)
    err = float(np.abs(got - ref).max())
    _say(f"  max |state - oracle| = {err:.2e}")
    assert err <= _tol(dtype), err


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_traj_path_agrees_with_per_stage_path(dtype):
    prob = cd.Problem(8, 8, 2, 1, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    a, b = _plan(prob, 9), _plan(prob, 9, "generic")
    assert a.path == 6 and b.path == 0
    ra = a.new_state()
    a.sample_noise(77, 0, ra)
    rb = ra.clone()
    a.step_rk4(ra, a.new_workspace(), 0.01, 20)
    b.step_rk4(rb, b.new_workspace(), 0.01, 20)
    torch.cuda.synchronize()
    diff = (ra - rb).abs().max().item()
    _say("traj vs per-stage, dtype", dtype, f"max diff {diff:.2e}")
    assert diff <= (1e-13 if dtype == cd.F64 else 2e-5)


def test_traj_zero_steps_and_single_trajectory():
    prob = cd.Problem(4, 4, 1, 1, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64)
    plan = _plan(prob, 1)
    assert plan.path == 6 and plan.resident == 1
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(5, 0, rho)
    before = rho.clone()
    plan.step_rk4(rho, ws, 0.01, 0)
    torch.cuda.synchronize()
    assert torch.equal(rho, before)
    plan.step_rk4(rho, ws, 0.05, 8)
    torch.cuda.synchronize()
    op = oracle.Problem(4, 4, 1, 1, d=3, periodic=True, J=1.0, U=5.0)
    _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=5, traj_offset=0, n_traj=1)
    err = float(np.abs(rho.cpu().numpy() - oracle.rk4(op, r0, 0.05, 8)).max())
    assert err <= 1e-12, err


def test_traj_schedule_runs_per_stage_and_matches_oracle():
    prob = cd.Problem(6, 6, 2, 1, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64)
    plan = _plan(prob, 3)
    assert plan.path == 6
    op = oracle.Problem(6, 6, 2, 1, d=3, periodic=True, J=1.0, U=5.0)
    n_steps, dt = 6, 0.02
    c1 = np.linspace(0.5, 1.5, 2 * n_steps + 1)
    c2 = np.linspace(8.0, 3.0, 2 * n_steps + 1)
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(31, 0, rho)
    plan.step_rk4_schedule(rho, ws, dt, n_steps, c1, c2)
    torch.cuda.synchronize()
    _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=31, traj_offset=0, n_traj=3)
    err = float(np.abs(rho.cpu().numpy() - oracle.rk4_schedule(op, r0, dt, n_steps, c1, c2)).max())
    assert err <= 1e-12, err


def test_traj_forced_where_it_cannot_run_is_rejected():
    with pytest.raises(cd.CdtwaError):
        _plan(cd.Problem(4, 4, 2, 2, d=3, dtype=cd.F64), 2, "traj")
    with pytest.raises(cd.CdtwaError):
        _plan(cd.Problem(4, 4, 1, 1, d=4, dtype=cd.F64), 2, "traj")
    with pytest.raises(cd.CdtwaError):   # one 48x48 trajectory of 1x1 FP64 clusters exceeds a workgroup
        _plan(cd.Problem(48, 48, 1, 1, d=3, dtype=cd.F64), 2, "traj")
    assert _plan(cd.Problem(48, 48, 1, 1, d=3, dtype=cd.F64), 2).path == 0


# lattices of the batching workload at their largest resident sizes: a few
# sampled trajectories of a many-block run against the oracle
@pytest.mark.parametrize("dtype,Lx,cx,cy", [(cd.F64, 16, 1, 1), (cd.F32, 24, 1, 1), (cd.F64, 8, 2, 1),
                                             (cd.F32, 8, 1, 2)])
def test_traj_workload_sizes_sampled_against_oracle(dtype, Lx, cx, cy):
    prob = cd.Problem(Lx, Lx, cx, cy, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    n = 1024
    plan = _plan(prob, n)
    assert plan.path == 6
    _say("traj workload", Lx, cx, cy, dtype, "per workgroup", plan.resident)
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(8, 0, rho)
    plan.step_rk4(rho, ws, 0.01, 25)
    torch.cuda.synchronize()
    op = oracle.Problem(Lx, Lx, cx, cy, d=3, periodic=True, J=1.0, U=5.0)
    for t in (0, plan.resident, n - 1):
        _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=8, traj_offset=t, n_traj=1)
        ref = oracle.rk4(op, r0, 0.01, 25)
        err = float(np.abs(rho[t:t + 1].cpu().numpy().astype(np.complex128) - ref).max())
        _say(f"  trajectory {t}: max |state - oracle| = {err:.2e}")
        assert err <= _tol(dtype), (t, err)
