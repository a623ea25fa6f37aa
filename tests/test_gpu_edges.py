"""Degenerate and boundary cases of the HIP path: zero RK4 steps (the state
is left bit for bit), invalid time steps (rejected before anything is
enqueued, the state untouched), decoupled clusters (J = 0: every cluster
evolves under its own interaction only) and the interaction-free lattice
(U = 0), on the fused and the per-stage paths, against the oracle."""
import math
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


def _plan(prob, n, path):
    old = os.environ.get("CDTWA_PATH")
    os.environ["CDTWA_PATH"] = path
    try:
        return cd.Plan(prob, n)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


@pytest.mark.parametrize("path,expect", [("fused27", 1), ("generic", 0)])
def test_zero_steps_leave_the_state_untouched(path, expect):
    prob = cd.Problem(4, 4, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64)
    plan = _plan(prob, 3, path)
    assert plan.path == expect
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(11, 0, rho)
    before = rho.clone()
    plan.step_rk4(rho, ws, 0.01, 0)
    torch.cuda.synchronize()
    assert torch.equal(rho, before)


@pytest.mark.parametrize("dt", [0.0, -0.01, math.nan, math.inf])
def test_invalid_time_steps_are_rejected(dt):
    prob = cd.Problem(4, 4, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64)
    plan = cd.Plan(prob, 2)
    rho, ws = plan.new_state(), plan.new_workspace()
    plan.sample_noise(12, 0, rho)
    before = rho.clone()
    with pytest.raises(cd.CdtwaError):
        plan.step_rk4(rho, ws, dt, 3)
    with pytest.raises(cd.CdtwaError):
        plan.step_rk4(rho, ws, 0.01, -1)
    torch.cuda.synchronize()
    assert torch.equal(rho, before)


@pytest.mark.parametrize("path,expect", [("fused27", 1), ("generic", 0)])
@pytest.mark.parametrize("J,U", [(0.0, 5.0), (1.0, 0.0)])
def test_decoupled_and_interaction_free(J, U, path, expect):
    """J = 0: the mean fields vanish and each cluster matrix only rotates
    under its diagonal interaction; U = 0: hopping and fields only."""
    _say("edges", J, U, path)
    prob = cd.Problem(4, 4, 2, 2, d=3, periodic=True, J=J, U=U, dtype=cd.F64)
    op = oracle.Problem(4, 4, 2, 2, d=3, periodic=True, J=J, U=U)
    n = 3
    _, rho0 = oracle.sample(op, oracle.mott_tables(3), seed=21, traj_offset=0, n_traj=n)
    plan = _plan(prob, n, path)
    assert plan.path == expect
    r = torch.from_numpy(rho0).cuda()
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.02, 10)
    torch.cuda.synchronize()
    ref = oracle.rk4(op, rho0, 0.02, 10)
    assert np.abs(r.cpu().numpy() - ref).max() < 1e-12
    if J == 0.0:
        # the interaction is diagonal in the occupation basis: populations stay put
        got = r.cpu().numpy()
        diag = np.diagonal(got, axis1=-2, axis2=-1)
        assert np.abs(diag - np.diagonal(rho0, axis1=-2, axis2=-1)).max() < 1e-12
