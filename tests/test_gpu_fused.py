"""The fused persistent RK4 kernels (2x2 clusters, d = 3: the 27-row kernel,
path 1, and the 9-row plaquette kernel, path 2) against the oracle and
against the per-stage path, including several trajectory rounds, ragged
trajectory counts and open boundaries."""
import os

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


PATHS = {"generic": 0, "fused27": 1, "plaq": 2, "dense": 3}


def _plan(prob, n, path):
    old = os.environ.get("CDTWA_PATH")
    try:
        os.environ["CDTWA_PATH"] = path
        return cd.Plan(prob, n)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


@pytest.mark.parametrize("path", ["fused27", "plaq"])
@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
@pytest.mark.parametrize("lat", [(4, 4, True), (8, 6, True), (4, 6, False), (6, 4, False)])
def test_fused_matches_oracle(lat, dtype, path):
    Lx, Ly, periodic = lat
    _say("fused vs oracle", lat, dtype, path)
    gp = cd.Problem(Lx, Ly, 2, 2, d=3, periodic=periodic, J=1.0, U=5.0, dtype=dtype)
    op = oracle.Problem(Lx, Ly, 2, 2, d=3, periodic=periodic, J=1.0, U=5.0)
    n = 3
    _, rho0 = oracle.sample(op, oracle.mott_tables(3), seed=8, traj_offset=0, n_traj=n)
    plan = _plan(gp, n, path)
    assert plan.path == PATHS[path], "fused path not selected"
    r = torch.from_numpy(rho0).to(gp.complex_dtype).cuda()
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.02, 15)
    assert plan.device_status(ws) == 0
    ref = oracle.rk4(op, rho0, 0.02, 15)
    err = np.abs(r.cpu().numpy() - ref).max()
    _say("max err", err)
    assert err < (1e-12 if dtype == cd.F64 else 2e-5)


@pytest.mark.parametrize("path", ["fused27", "plaq"])
@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_fused_equals_generic_over_rounds(dtype, path):
    """More trajectories than fit at once (several rounds), odd count."""
    gp = cd.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    fused = _plan(gp, 7, path)
    generic = _plan(gp, 7, "generic")
    _say("fused vs generic 32x32", dtype, path, "resident", fused.resident)
    assert fused.path == PATHS[path] and generic.path == 0
    assert fused.resident < 7
    rho = fused.new_state()
    fused.sample_noise(42, 0, rho)
    r2 = rho.clone()
    wf, wg = fused.new_workspace(), generic.new_workspace()
    for _ in range(3):          # three calls: tags restart every call
        fused.step_rk4(rho, wf, 0.01, 4)
        generic.step_rk4(r2, wg, 0.01, 4)
    assert fused.device_status(wf) == 0
    err = (rho - r2).abs().max().item()
    _say("max |fused - generic|", err)
    assert err < (1e-12 if dtype == cd.F64 else 1e-5)


@pytest.mark.parametrize("lat", [(4, 4, True), (6, 4, False)])
def test_dense_mfma_path_matches_oracle(lat):
    """Path 3: M = H Y as a dense complex product on the matrix cores (FP32)."""
    Lx, Ly, periodic = lat
    _say("dense path vs oracle", lat)
    gp = cd.Problem(Lx, Ly, 2, 2, d=3, periodic=periodic, J=1.0, U=5.0, dtype=cd.F32)
    op = oracle.Problem(Lx, Ly, 2, 2, d=3, periodic=periodic, J=1.0, U=5.0)
    n = 3
    _, rho0 = oracle.sample(op, oracle.mott_tables(3), seed=8, traj_offset=0, n_traj=n)
    plan = _plan(gp, n, "dense")
    assert plan.path == 3
    r = torch.from_numpy(rho0).to(torch.complex64).cuda()
    ws = plan.new_workspace()
    K = plan.new_state()
    plan.commutator(r, K, ws)
    Kref = oracle.rhs(op, rho0)
    assert np.abs(K.cpu().numpy() - Kref).max() < 2e-5 * np.abs(Kref).max()
    plan.step_rk4(r, ws, 0.02, 15)
    ref = oracle.rk4(op, rho0, 0.02, 15)
    err = np.abs(r.cpu().numpy() - ref).max()
    _say("max err", err)
    assert err < 2e-5


def test_dense_path_rejects_fp64():
    gp = cd.Problem(4, 4, 2, 2, d=3, dtype=cd.F64)
    with pytest.raises(cd.CdtwaError):
        _plan(gp, 2, "dense")


@pytest.mark.parametrize("path,dtype", [("fused27", cd.F64), ("plaq", cd.F32)])
def test_neighbour_wait_timeout_is_reported(path, dtype):
    """A spin limit of 0 polls makes the fused kernels' neighbour waits time
    out: every workgroup still exits, the status word reports it and the
    affected clusters hold NaN; the next call on a normal plan is clean."""
    gp = cd.Problem(32, 32, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=dtype)
    old = os.environ.get("CDTWA_SPIN_LIMIT")
    os.environ["CDTWA_SPIN_LIMIT"] = "0"
    try:
        plan = _plan(gp, 3, path)
    finally:
        if old is None:
            os.environ.pop("CDTWA_SPIN_LIMIT", None)
        else:
            os.environ["CDTWA_SPIN_LIMIT"] = old
    _say("timeout path", path, dtype)
    rho = plan.new_state()
    plan.sample_noise(9, 0, rho)
    ws = plan.new_workspace()
    plan.step_rk4(rho, ws, 0.01, 10)
    status = plan.device_status(ws)
    finite = bool(torch.isfinite(torch.view_as_real(rho)).all())
    _say("status", status, "finite", finite)
    assert status in (0, 1)
    # every cluster and stage finding all neighbour words at the first look
    # is possible in principle; then nothing may have been poisoned
    assert (status == 1) == (not finite)
    normal = _plan(gp, 3, path)
    r2 = normal.new_state()
    normal.sample_noise(9, 0, r2)
    w2 = normal.new_workspace()
    normal.step_rk4(r2, w2, 0.01, 10)
    assert normal.device_status(w2) == 0
    assert torch.isfinite(torch.view_as_real(r2)).all()

def test_wide_fp32_build_for_lattices_beyond_two_workgroups_per_cu():
    """48x48 lattice, 2x2 clusters (576 clusters, more than two workgroups
    per CU hold): FP32 plans take the fused kernel built for three workgroups
    per CU; against the oracle on two trajectories (one at a time) and
    against the per-stage path on five."""
    gp = cd.Problem(48, 48, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F32)
    op = oracle.Problem(48, 48, 2, 2, d=3, periodic=True, J=1.0, U=5.0)
    plan = cd.Plan(gp, 2)
    _say("wide fp32 48x48: path", plan.path, "resident", plan.resident)
    assert plan.path == 1 and plan.resident == 1
    _, rho0 = oracle.sample(op, oracle.mott_tables(3), seed=5, traj_offset=0, n_traj=2)
    r = torch.from_numpy(rho0).to(gp.complex_dtype).cuda()
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.01, 4)
    assert plan.device_status(ws) == 0
    err = np.abs(r.cpu().numpy() - oracle.rk4(op, rho0, 0.01, 4)).max()
    _say("max err vs oracle", err)
    assert err < 2e-5
    fused, generic = cd.Plan(gp, 5), _plan(gp, 5, "generic")
    assert fused.path == 1 and generic.path == 0
    a = fused.new_state()
    fused.sample_noise(3, 0, a)
    b = a.clone()
    fused.step_rk4(a, fused.new_workspace(), 0.01, 6)
    generic.step_rk4(b, generic.new_workspace(), 0.01, 6)
    err = (a - b).abs().max().item()
    _say("max |fused - generic|", err)
    assert err < 1e-5
    # FP64 and open systems keep the per-stage path at this size
    assert cd.Plan(cd.Problem(48, 48, 2, 2, d=3, periodic=True, dtype=cd.F64), 2).path == 0
