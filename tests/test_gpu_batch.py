"""Problem batches (cdtwa_batch_*): one persistent trajectory-resident
launch for every member on that path, one cooperative launch of the fused
kernel for the 2x2 members on the fused path (gangs of several members
side by side), one mixed-shape launch per RK4 stage for the other d = 3
members of the per-stage launch (graph-captured steps, autotuned workgroup
shapes).  Every member must end bit for bit where its own plan's
cdtwa_step_rk4 takes it: the resident and fused launches run each member's
trajectories exactly as its own plan does, the mixed kernel runs the same
per-cluster arithmetic as the per-stage kernel, and the remaining members
run their own path.  Every member (each cluster shape, d = 2, 3, 4, resident,
mixed and own-path) is also compared with the FP64 oracle on the same
noise, entry by entry."""
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


# (Lx, Ly, cx, cy, d, U, n_traj, path)
MEMBERS = [
    (8, 8, 1, 1, 3, 3.0, 64, None),        # resident
    (8, 8, 2, 1, 3, 5.0, 32, None),        # resident
    (8, 8, 1, 2, 3, 10.0, 16, None),       # resident
    (16, 16, 1, 1, 3, 5.0, 8, None),       # resident
    (6, 6, 2, 1, 3, 3.0, 5, "generic"),    # small clusters on the per-stage path: mixed
    (48, 48, 1, 1, 3, 5.0, 2, None),       # a trajectory too large for a workgroup: mixed
    (4, 4, 2, 2, 3, 5.0, 5, "generic"),    # 2x2 on the per-stage path: mixed
    (8, 8, 2, 2, 3, 3.0, 3, None),         # fused path: the batch's fused launch unless mix_all
    (12, 8, 2, 2, 3, 10.0, 6, None),       # fused path, 24 clusters: the same fused launch
    (6, 4, 1, 1, 4, 5.0, 4, None),         # d = 4: own path
    (4, 4, 2, 2, 2, 5.0, 4, None),         # d = 2: own path
]


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
@pytest.mark.parametrize("mix_all", [False, True])
def test_batch_matches_each_plan(dtype, mix_all):
    _say("batch", dtype, "mix_all", mix_all)
    plans, refs, rhos, ref_rhos = [], [], [], []
    for i, (Lx, Ly, cx, cy, d, U, n, path) in enumerate(MEMBERS):
        prob = cd.Problem(Lx, Ly, cx, cy, d=d, periodic=True, J=1.0, U=U, dtype=dtype)
        p = _plan(prob, n, path)
        # the reference of a member that enters the mixed launch is the
        # per-stage path; the others run their own path in both
        mixed = d == 3 and p.path != 6 and (cx * cy < 4 or path == "generic" or mix_all)
        r = _plan(prob, n, "generic" if mixed else path)
        rho = p.new_state()
        p.sample_noise(100 + i, 7, rho)
        plans.append(p)
        refs.append(r)
        rhos.append(rho)
        ref_rhos.append(rho.clone())
    batch = cd.Batch(plans, mix_all=mix_all)
    ws = batch.new_workspaces()
    ref_ws = [r.new_workspace() for r in refs]
    batch.step_rk4(rhos, ws, 0.01, 5)
    info = batch.info()
    _say("  info", info)
    assert info["mixed_members"] == (5 if mix_all else 3)
    assert info["resident_members"] == 4 and info["resident_items"] >= 4
    assert info["fused_members"] == (0 if mix_all else 2)
    assert info["threads"] in (512, 1024)
    batch.step_rk4(rhos, ws, 0.02, 3)                # new dt: the graph is captured again
    moved = [r.clone() for r in rhos]                # new pointers: the tables are rewritten
    batch.step_rk4(moved, ws, 0.02, 2)
    for r, rr, w in zip(refs, ref_rhos, ref_ws):
        r.step_rk4(rr, w, 0.01, 5)
        r.step_rk4(rr, w, 0.02, 3)
        r.step_rk4(rr, w, 0.02, 2)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(moved, ref_rhos)):
        assert torch.isfinite(torch.view_as_real(a)).all(), i
        assert torch.equal(a, b), (i, MEMBERS[i], (a - b).abs().max().item())
    # every member against the oracle: same noise, the same three calls
    tol = 1e-12 if dtype == cd.F64 else 2e-5
    for i, (Lx, Ly, cx, cy, d, U, n, path) in enumerate(MEMBERS):
        op = oracle.Problem(Lx, Ly, cx, cy, d=d, periodic=True, J=1.0, U=U)
        _, r0 = oracle.sample(op, oracle.mott_tables(d), seed=100 + i, traj_offset=7, n_traj=n)
        r1 = oracle.rk4(op, oracle.rk4(op, r0, 0.01, 5), 0.02, 5)
        err = float(np.abs(moved[i].cpu().numpy().astype(np.complex128) - r1).max())
        _say(f"  member {i} {MEMBERS[i][:5]}: max |state - oracle| = {err:.2e}")
        assert err <= tol, (i, MEMBERS[i], err)


def test_batch_rejects_mixed_precision():
    a = cd.Plan(cd.Problem(4, 4, 1, 1, d=3, dtype=cd.F64), 2)
    b = cd.Plan(cd.Problem(4, 4, 1, 1, d=3, dtype=cd.F32), 2)
    with pytest.raises(cd.CdtwaError):
        cd.Batch([a, b])


# members of the batching workload's kinds at sizes the oracle integrates to
# T = 4/J in seconds: resident (1x1, 2x1, 1x2 on 8x8), per-stage mixed (2x1
# on 16x16, 1x1 on 48x48: trajectories too large for a workgroup), the
# fused launch (2x2 on 8x8 and 4x4)
T4_MEMBERS = [
    (8, 8, 1, 1, 3.0, 40), (8, 8, 2, 1, 5.0, 12), (8, 8, 1, 2, 10.0, 12),
    (16, 16, 2, 1, 3.0, 4), (48, 48, 1, 1, 5.0, 2),
    (8, 8, 2, 2, 10.0, 3), (4, 4, 2, 2, 3.0, 4),
]


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_batch_to_T4(dtype):
    """One batch call of 400 steps (dt = 0.01/J, T = 4/J).  Every member ends
    bit for bit where its own plan's cdtwa_step_rk4 takes it (per-stage path
    for the members of the mixed launch).  FP64: the first and last
    trajectory of every member within 1e-10 of the oracle.  (FP32 entries
    carry rounding amplified through 400 steps of the mean-field dynamics;
    the 1e-5 target of the FP32 state is stated on sample means and asserted
    there.)"""
    _say("batch to T = 4/J, dtype", dtype)
    plans, refs, rhos, ref_rhos = [], [], [], []
    for i, (Lx, Ly, cx, cy, U, n) in enumerate(T4_MEMBERS):
        prob = cd.Problem(Lx, Ly, cx, cy, d=3, periodic=True, J=1.0, U=U, dtype=dtype)
        p = cd.Plan(prob, n)
        r = p.new_state()
        p.sample_noise(300 + i, 0, r)
        plans.append(p)
        rhos.append(r)
        ref_rhos.append(r.clone())
        refs.append(_plan(prob, n, "generic" if p.path == 0 else None))
    _say("  paths", [p.path for p in plans])
    assert [p.path for p in plans][:5] == [6, 6, 6, 0, 0]
    batch = cd.Batch(plans)
    ws = batch.new_workspaces()
    batch.step_rk4(rhos, ws, 0.01, 400)
    for r, rr in zip(refs, ref_rhos):
        r.step_rk4(rr, r.new_workspace(), 0.01, 400)
    torch.cuda.synchronize()
    info = batch.info()
    assert info["resident_members"] == 3 and info["mixed_members"] == 2 and info["fused_members"] == 2
    for i, (a, b) in enumerate(zip(rhos, ref_rhos)):
        assert torch.isfinite(torch.view_as_real(a)).all(), i
        assert torch.equal(a, b), (i, T4_MEMBERS[i], (a - b).abs().max().item())
    if dtype == cd.F64:
        for i, (Lx, Ly, cx, cy, U, n) in enumerate(T4_MEMBERS):
            op = oracle.Problem(Lx, Ly, cx, cy, d=3, periodic=True, J=1.0, U=U)
            for t in (0, n - 1):
                _, r0 = oracle.sample(op, oracle.mott_tables(3), seed=300 + i, traj_offset=t, n_traj=1)
                ref = oracle.rk4(op, r0, 0.01, 400)
                err = float(np.abs(rhos[i][t:t + 1].cpu().numpy() - ref).max())
                _say(f"  member {T4_MEMBERS[i]} path {plans[i].path} trajectory {t}: "
                     f"max |state - oracle| = {err:.2e}")
                assert err <= 1e-10, (i, t, err)
    batch.close()
