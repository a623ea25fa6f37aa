"""Parity at the benchmark's full size and launch configuration: the 32x32
periodic lattice, 256 clusters of 2x2 sites, d = 3, U/J = 5, dt = 0.01,
calls of 10 RK4 steps on the default fused path (the 27-row kernel; one
trajectory resident at a time in FP64, two in FP32, so several trajectory
rounds per call), observables recorded after every call.  A few
trajectories, checked against the oracle on every recorded observable and,
for FP64, on the whole final state."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_benchmark_configuration_matches_oracle(dtype):
    n, calls, every = 3, 3, 10
    gp = cd.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    op = oracle.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0)
    plan = cd.Plan(gp, n)
    print("32x32 benchmark configuration, dtype", dtype, "path", plan.path, "resident", plan.resident, flush=True)
    assert plan.path == 1
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(2024, 500, rho)
    sums = torch.zeros(calls + 1, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(calls + 1, n, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(rho, 0, sums, ws, per_traj=per[0])
    for k in range(calls):
        plan.step_rk4(rho, ws, 0.01, every)
        plan.accumulate_observables(rho, k + 1, sums, ws, per_traj=per[k + 1])
    assert plan.device_status(ws) == 0
    torch.cuda.synchronize()
    res = oracle.run(op, oracle.mott_tables(3), seed=2024, traj_offset=500, n_traj=n, dt=0.01, n_steps=calls * every,
                     record_steps=[k * every for k in range(calls + 1)], want_rho=(dtype == cd.F64))
    got = per.cpu().numpy().transpose(1, 0, 2)
    err = np.abs(got[:, :, :12] - res["obs"][:, :, :12]).max()
    print("max observable error", err, flush=True)
    if dtype == cd.F64:
        assert err < 1e-11
        serr = np.abs(rho.cpu().numpy() - res["rho"]).max()
        print("max state error", serr, flush=True)
        assert serr < 1e-12
    else:
        assert err < 2e-5


# The benchmark's timed batch: 1024 trajectories per call (1024 trajectory
# rounds of the persistent kernel per call in FP64, 512 in FP32),
# observables after every call of 10 steps.  Three trajectories spread over the batch are run
# through the oracle one by one and compared; the sums over the whole batch
# are checked against the per-trajectory records.
BATCH = 1024
SAMPLE = (0, 517, 1023)


@pytest.fixture(scope="module")
def batch_oracle():
    op = oracle.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0)
    return {i: oracle.run(op, oracle.mott_tables(3), seed=77, traj_offset=9000 + i, n_traj=1, dt=0.01, n_steps=20,
                          record_steps=[0, 10, 20], want_rho=True) for i in SAMPLE}


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_benchmark_batch_sampled_against_oracle(dtype, batch_oracle):
    gp = cd.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    plan = cd.Plan(gp, BATCH)
    print("32x32 batch of", BATCH, "dtype", dtype, "path", plan.path, "resident", plan.resident, flush=True)
    assert plan.path == 1
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(77, 9000, rho)
    sums = torch.zeros(3, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(3, BATCH, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(rho, 0, sums, ws, per_traj=per[0])
    for k in range(2):
        plan.step_rk4(rho, ws, 0.01, 10)
        plan.accumulate_observables(rho, k + 1, sums, ws, per_traj=per[k + 1])
    assert plan.device_status(ws) == 0
    torch.cuda.synchronize()
    got = per.cpu().numpy()                                  # [n_rec][BATCH][NOBS]
    assert np.isfinite(got).all()
    for i in SAMPLE:
        ref = batch_oracle[i]
        err = np.abs(got[:, i, :12] - ref["obs"][0, :, :12]).max()
        print("trajectory", i, "max observable error", err, flush=True)
        if dtype == cd.F64:
            assert err < 1e-11
            serr = np.abs(rho[i].cpu().numpy() - ref["rho"][0]).max()
            print("trajectory", i, "max state error", serr, flush=True)
            assert serr < 1e-12
        else:
            assert err < 2e-5
    s = sums.cpu().numpy()
    assert np.allclose(s[:, :, 0] + s[:, :, 1], got.sum(axis=1), rtol=1e-12, atol=1e-12)
    assert np.allclose(s[:, :, 2], (got ** 2).sum(axis=1), rtol=1e-12, atol=1e-12)


# The D = 256 path at the size of its benchmark leg: 16x16 periodic lattice,
# 2x2 clusters with d = 4, 256 trajectories in one call (three launches per
# stage over every cluster of the batch), trajectories 0, 101 and 255 against
# the oracle one by one.
D256_BATCH = 256
D256_SAMPLE = (0, 101, 255)


@pytest.fixture(scope="module")
def d256_oracle():
    op = oracle.Problem(16, 16, 2, 2, d=4, periodic=True, J=1.0, U=5.0)
    return {i: oracle.run(op, oracle.mott_tables(4), seed=11, traj_offset=i, n_traj=1, dt=0.01, n_steps=8,
                          record_steps=[0, 8], want_rho=True) for i in D256_SAMPLE}


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_d256_batch_sampled_against_oracle(dtype, d256_oracle):
    gp = cd.Problem(16, 16, 2, 2, d=4, periodic=True, J=1.0, U=5.0, dtype=dtype)
    plan = cd.Plan(gp, D256_BATCH)
    print("16x16 d=4 batch of", D256_BATCH, "dtype", dtype, "path", plan.path, flush=True)
    assert plan.path == 0 and plan.D == 256
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(11, 0, rho)
    sums = torch.zeros(2, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(2, D256_BATCH, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(rho, 0, sums, ws, per_traj=per[0])
    plan.step_rk4(rho, ws, 0.01, 8)
    plan.accumulate_observables(rho, 1, sums, ws, per_traj=per[1])
    torch.cuda.synchronize()
    got = per.cpu().numpy()
    assert np.isfinite(got).all()
    for i in D256_SAMPLE:
        ref = d256_oracle[i]
        err = np.abs(got[:, i, :12] - ref["obs"][0, :, :12]).max()
        print("trajectory", i, "max observable error", err, flush=True)
        if dtype == cd.F64:
            assert err < 1e-11
            serr = np.abs(rho[i].cpu().numpy() - ref["rho"][0]).max()
            print("trajectory", i, "max state error", serr, flush=True)
            assert serr < 1e-12
        else:
            assert err < 2e-5


# The batching workload at full size, in the launch configuration the
# benchmark times: 36 instances (1x1, 2x1, 2x2 clusters x sides 8, 16, 24, 48
# x U/J 3, 5, 10; 4096, 2048, 1024, 256 trajectories), FP32 state, one batch
# call.  Its small-cluster members that fit a workgroup go to the
# trajectory-resident launch, the others to the per-stage mixed launch, the
# 2x2 members to their fused launches.  After two RK4 steps the first and the
# last trajectory of every member are run through the oracle one by one.
def test_batching_workload_sampled_against_oracle():
    traj = {8: 4096, 16: 2048, 24: 1024, 48: 256}
    members = [(L, cx, cy, U) for (cx, cy) in ((1, 1), (2, 1), (2, 2)) for L in (8, 16, 24, 48)
               for U in (3.0, 5.0, 10.0)]
    plans, rhos = [], []
    for i, (L, cx, cy, U) in enumerate(members):
        p = cd.Plan(cd.Problem(L, L, cx, cy, d=3, periodic=True, J=1.0, U=U, dtype=cd.F32), traj[L])
        r = p.new_state()
        p.sample_noise(900 + i, 0, r)
        plans.append(p)
        rhos.append(r)
    batch = cd.Batch(plans)
    ws = batch.new_workspaces()
    batch.step_rk4(rhos, ws, 0.01, 2)
    torch.cuda.synchronize()
    info = batch.info()
    print("batching workload:", info, "paths", [p.path for p in plans], flush=True)
    assert info["resident_members"] == 12 and info["mixed_members"] == 12
    worst = 0.0
    for i, (L, cx, cy, U) in enumerate(members):
        op = oracle.Problem(L, L, cx, cy, d=3, periodic=True, J=1.0, U=U)
        for t in (0, traj[L] - 1):
            _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=900 + i, traj_offset=t, n_traj=1)
            ref = oracle.rk4(op, r0, 0.01, 2)
            err = float(np.abs(rhos[i][t:t + 1].cpu().numpy().astype(np.complex128) - ref).max())
            worst = max(worst, err)
            assert err < 2e-5, (members[i], t, err)
    print("worst |state - oracle| over the sampled trajectories:", worst, flush=True)
    batch.close()
    for p in plans:
        p.close()
