"""Open-system extension on the GPU (local Lindblad channels L = n_j and
L = a_j on every cluster matrix) against the oracle: the right-hand side
(commutator plus dissipator), RK4 steps on the per-stage path and on the
fused 27-row path (2x2 clusters, d = 3), several trajectory rounds of the
fused kernel, a time-dependent schedule, FP32 quenches, the 32x32 lattice
of the benchmark, and the plan rules."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


SHAPES = [
    # (Lx, Ly, cx, cy, d, periodic, gdeph, gloss)
    (4, 4, 2, 2, 3, True, 0.5, 0.3),
    (4, 6, 2, 2, 3, False, 0.0, 0.8),
    (6, 4, 2, 1, 3, True, 0.7, 0.0),
    (4, 4, 1, 2, 4, True, 0.2, 0.4),
    (3, 3, 1, 1, 4, True, 0.6, 0.6),
    (4, 4, 2, 2, 2, False, 0.3, 0.9),
]


def _probs(Lx, Ly, cx, cy, d, periodic, gd, gl, dtype=cd.F64):
    return (cd.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=1.0, U=5.0, dtype=dtype, gamma_deph=gd,
                       gamma_loss=gl),
            oracle.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=1.0, U=5.0, gdeph=gd, gloss=gl))


def _state(op, d, n):
    closed = oracle.Problem(op.Lx, op.Ly, op.cx, op.cy, d=d, periodic=op.periodic, J=1.0, U=5.0)
    _, rho = oracle.sample(closed, oracle.mott_tables(d), seed=13, traj_offset=0, n_traj=n)
    return oracle.rk4(op, rho, 0.05, 3)


@pytest.mark.parametrize("shape", SHAPES)
def test_lindblad_rhs_and_rk4(shape):
    gp, op = _probs(*shape)
    _say("lindblad", shape)
    n = 3
    rho = _state(op, shape[4], n)
    plan = cd.Plan(gp, n)
    assert plan.path == (1 if shape[2:5] == (2, 2, 3) else 0)
    r = torch.from_numpy(rho).cuda()
    ws = plan.new_workspace()
    K = plan.new_state()
    plan.commutator(r, K, ws)
    torch.cuda.synchronize()
    Kref = oracle.rhs(op, rho)
    assert np.abs(K.cpu().numpy() - Kref).max() < 1e-13 * max(np.abs(Kref).max(), 1.0)
    plan.step_rk4(r, ws, 0.02, 9)
    torch.cuda.synchronize()
    assert np.abs(r.cpu().numpy() - oracle.rk4(op, rho, 0.02, 9)).max() < 1e-12


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_lindblad_fp32_quench_and_schedule(shape):
    gp, op = _probs(*shape, dtype=cd.F32)
    _say("lindblad fp32/schedule", shape)
    rec = [0, 6, 12]
    sums, per = cd.run_quench(gp, 5, seed=2, dt=0.025, record_steps=rec)
    ref = oracle.run(op, oracle.mott_tables(shape[4]), seed=2, traj_offset=0, n_traj=5, dt=0.025, n_steps=12,
                     record_steps=rec)["obs"]
    assert np.abs(per.numpy()[:, :, :12] - ref[:, :, :12]).max() < 2e-5
    # schedule on an FP64 plan of the same open system
    g64, _ = _probs(*shape)
    n, steps, dt = 2, 20, 0.02
    rho = _state(op, shape[4], n)
    plan = cd.Plan(g64, n)
    r = torch.from_numpy(rho).cuda()
    ws = plan.new_workspace()
    th = 0.5 * dt * np.arange(2 * steps + 1)
    c1, c2 = 1.0 + 0.3 * np.cos(4 * th), 5.0 - 10.0 * th
    plan.step_rk4_schedule(r, ws, dt, steps, c1, c2)
    torch.cuda.synchronize()
    assert np.abs(r.cpu().numpy() - oracle.rk4_schedule(op, rho, dt, steps, c1, c2)).max() < 1e-12


def _forced(path, fn):
    old = os.environ.get("CDTWA_PATH")
    os.environ["CDTWA_PATH"] = path
    try:
        return fn()
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_lindblad_fused_rounds(dtype):
    """More trajectories than the chip holds at once (the fused kernel runs
    them in rounds, refilling the triangle of Y for each), against the oracle
    and against the per-stage path."""
    shape = (4, 4, 2, 2, 3, True, 0.4, 0.25)
    gp, op = _probs(*shape, dtype=dtype)
    n = cd.Plan(gp, 100000).resident + 6
    plan = cd.Plan(gp, n)
    assert plan.path == 1 and plan.resident < n
    _say("lindblad fused rounds", dtype, "trajectories", n, "resident", plan.resident)
    rho = _state(op, 3, n)
    ref = oracle.rk4(op, rho, 0.02, 6)
    tol = 1e-12 if dtype == cd.F64 else 3e-5
    r = torch.from_numpy(rho).to(gp.complex_dtype).cuda()
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.02, 6)
    torch.cuda.synchronize()
    assert plan.device_status(ws) == 0
    got = r.cpu().numpy()
    err = np.abs(got - ref).max()
    _say("max err vs oracle", err)
    assert err < tol
    # the per-stage path on the same input
    gen = _forced("generic", lambda: cd.Plan(gp, n))
    assert gen.path == 0
    r2 = torch.from_numpy(rho).to(gp.complex_dtype).cuda()
    gen.step_rk4(r2, gen.new_workspace(), 0.02, 6)
    torch.cuda.synchronize()
    assert np.abs(got - r2.cpu().numpy()).max() < tol


def test_lindblad_fused_benchmark_lattice():
    """The open-system benchmark lattice (32x32, 2x2 clusters, d = 3, FP64,
    dephasing 0.1, loss 0.05) on the fused path: two trajectories, five RK4
    steps, every cluster against the oracle."""
    shape = (32, 32, 2, 2, 3, True, 0.1, 0.05)
    gp, op = _probs(*shape)
    n = 2
    plan = cd.Plan(gp, n)
    assert plan.path == 1
    rho = _state(op, 3, n)
    r = torch.from_numpy(rho).cuda()
    plan.step_rk4(r, plan.new_workspace(), 0.01, 5)
    torch.cuda.synchronize()
    assert np.abs(r.cpu().numpy() - oracle.rk4(op, rho, 0.01, 5)).max() < 1e-12


def test_lindblad_plan_rules():
    gp, _ = _probs(4, 4, 2, 2, 3, True, 0.1, 0.1)
    old = os.environ.get("CDTWA_PATH")
    try:
        os.environ["CDTWA_PATH"] = "fused27"
        assert cd.Plan(gp, 2).path == 1
        for other in ("plaq", "dense", "spin"):
            os.environ["CDTWA_PATH"] = other
            with pytest.raises(cd.CdtwaError):
                cd.Plan(gp, 2)
        os.environ["CDTWA_PATH"] = "generic"
        assert cd.Plan(gp, 2).path == 0
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old
    with pytest.raises(cd.CdtwaError):      # D = 256 has no dissipator kernel
        cd.Plan(cd.Problem(4, 4, 2, 2, d=4, gamma_loss=0.1), 2)
