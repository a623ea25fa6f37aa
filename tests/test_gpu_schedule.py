"""Time-dependent couplings (cdtwa_step_rk4_schedule) on every path against
the oracle's RK4 with the same half-step schedule, and a constant schedule
against cdtwa_step_rk4 (to rounding).  37 steps, so that the fused paths run three
launches (16 + 16 + 5 steps) with the schedule in their kernel arguments."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")

N_STEPS, DT = 37, 0.01


def _say(*a):
    print(*a, flush=True)


def _plan(prob, n, path):
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


def _sched(n, c1=lambda t: 1.0 + 0.4 * np.sin(5.0 * t), c2=lambda t: 8.0 - 20.0 * t):
    t = 0.5 * DT * np.arange(2 * n + 1)
    return c1(t), c2(t)


# (label, path, Lx, Ly, cx, cy, d, periodic, dtype, model, expected path id)
CASES = [
    ("fused27-f64", "fused27", 4, 4, 2, 2, 3, True, cd.F64, 0, 1),
    ("fused27-f32", "fused27", 4, 6, 2, 2, 3, False, cd.F32, 0, 1),
    ("plaq-f32", "plaq", 4, 4, 2, 2, 3, True, cd.F32, 0, 2),
    ("plaq-f64", "plaq", 6, 4, 2, 2, 3, False, cd.F64, 0, 2),
    ("generic-2x2", "generic", 4, 4, 2, 2, 3, True, cd.F64, 0, 0),
    ("generic-1x1", "generic", 4, 6, 1, 1, 3, True, cd.F64, 0, 0),
    ("traj-1x1", None, 4, 6, 1, 1, 3, True, cd.F64, 0, 6),         # trajectory-resident plan: per-stage kernels
    ("traj-2x1-f32", None, 4, 4, 2, 1, 3, False, cd.F32, 0, 6),
    ("generic-2x1-d4", None, 4, 4, 2, 1, 4, True, cd.F64, 0, 0),
    ("big-d4", None, 4, 4, 2, 2, 4, True, cd.F64, 0, 0),
    ("dense-f32", "dense", 4, 4, 2, 2, 3, True, cd.F32, 0, 3),
    ("spinfused-2x2", None, 4, 4, 2, 2, 2, True, cd.F64, 1, 5),
    ("spinfused-2x2-f32", None, 4, 6, 2, 2, 2, False, cd.F32, 1, 5),
    ("spin-2x2", "spin", 4, 4, 2, 2, 2, True, cd.F64, 1, 4),
    ("spin-2x1", None, 4, 4, 2, 1, 2, True, cd.F64, 1, 4),
]


def _problems(case):
    _, path, Lx, Ly, cx, cy, d, periodic, dtype, model, _ = case
    kw = dict(model=1, h=1.0, init_state=1, U=0.0) if model == 1 else dict(U=5.0)
    return (cd.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=1.0, dtype=dtype, **kw),
            oracle.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=1.0, **kw))


def _tables(op, model, d):
    return oracle.neel_tables() if model == 1 else oracle.mott_tables(d)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_schedule_matches_oracle(case):
    label, path, *_rest = case
    model, want_path, d, dtype = case[9], case[10], case[6], case[8]
    gp, op = _problems(case)
    _say("schedule", label)
    n = 3
    _, rho0 = oracle.sample(op, _tables(op, model, d), seed=21, traj_offset=0, n_traj=n)
    rho0 = oracle.rk4(op, rho0, DT, 2)
    plan = _plan(gp, n, path)
    assert plan.path == want_path
    r = torch.from_numpy(rho0).to(gp.complex_dtype).cuda()
    ws = plan.new_workspace()
    c1, c2 = _sched(N_STEPS, c2=(lambda t: 1.5 - 3.0 * t) if model == 1 else (lambda t: 8.0 - 20.0 * t))
    plan.step_rk4_schedule(r, ws, DT, N_STEPS, c1, c2)
    assert plan.device_status(ws) == 0
    ref = oracle.rk4_schedule(op, rho0, DT, N_STEPS, c1, c2)
    if dtype == cd.F64:
        err = np.abs(r.cpu().numpy() - ref).max()
        _say("max err", err)
        assert err < 1e-11
    else:
        got = oracle.observables(op, r.cpu().numpy().astype(np.complex128))
        err = np.abs(got[:, :12] - oracle.observables(op, ref)[:, :12]).max()
        _say("max obs err", err)
        assert err < 2e-5


@pytest.mark.parametrize("path,dtype", [("fused27", cd.F64), ("plaq", cd.F32), ("generic", cd.F64)])
def test_constant_schedule_equals_step_rk4(path, dtype):
    gp = cd.Problem(8, 4, 2, 2, d=3, periodic=True, J=0.9, U=4.0, dtype=dtype)
    _say("constant schedule", path, dtype)
    n = 5
    plan = _plan(gp, n, path)
    a = plan.new_state()
    plan.sample_noise(5, 0, a)
    b = a.clone()
    wa, wb = plan.new_workspace(), plan.new_workspace()
    plan.step_rk4(a, wa, DT, N_STEPS)
    plan.step_rk4_schedule(b, wb, DT, N_STEPS, [0.9] * (2 * N_STEPS + 1), [4.0] * (2 * N_STEPS + 1))
    torch.cuda.synchronize()
    # the same arithmetic up to where the compiler contracts multiply-adds
    # around the per-stage coupling loads: equal to rounding
    err = (a - b).abs().max().item()
    _say("max diff", err)
    assert err < (1e-12 if dtype == cd.F64 else 1e-5)


def test_schedule_rejects_bad_input():
    gp = cd.Problem(4, 4, 2, 2, d=3, periodic=True)
    plan = cd.Plan(gp, 1)
    r, ws = plan.new_state(), plan.new_workspace()
    with pytest.raises(cd.CdtwaError):
        plan.step_rk4_schedule(r, ws, DT, 2, [1.0] * 4, [5.0] * 4)           # 2 n + 1 values needed
    with pytest.raises(cd.CdtwaError):
        plan.step_rk4_schedule(r, ws, DT, 2, [1.0, float("nan"), 1, 1, 1], [5.0] * 5)
