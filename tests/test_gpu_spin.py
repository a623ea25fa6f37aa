"""Transverse-field Ising model (App. A Eq. (Hising)) on the HIP spin paths
(plan path 5, the fused kernel for 2x2 clusters, and path 4, the per-stage
kernels) against the FP64 oracle, entry point by entry point and for whole
quenches, the fused kernel against the per-stage kernels over several
trajectory rounds, its wait timeout, and the four-site chain of App. A
against exact diagonalisation.

Tolerances as for the Bose-Hubbard parity tests: FP64 single stages at 1e-13
relative to the largest entry, trajectories at 1e-10 absolute; FP32 within
2e-5 absolute on O(1) observables over short runs.
"""
import itertools
import os

import numpy as np
import pytest
import torch

import oracle
from exact import evolve, ising_hamiltonian, spin_op, spin_product_state

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


SHAPES = [
    # (Lx, Ly, cx, cy, periodic, init_state)
    (4, 1, 2, 1, False, 1),     # the four-site chain of App. A, two-site clusters
    (4, 1, 1, 1, False, 1),
    (6, 1, 2, 1, False, 0),
    (4, 4, 2, 2, True, 1),
    (4, 4, 1, 2, False, 1),
    (6, 4, 2, 1, True, 0),
    (3, 3, 1, 1, True, 1),
    (4, 6, 2, 2, False, 1),
]
J, H = 1.0, 0.7


def _probs(Lx, Ly, cx, cy, periodic, init, dtype=1, J=J, h=H):
    return (cd.Problem(Lx, Ly, cx, cy, d=2, periodic=periodic, J=J, U=0.0, dtype=dtype, model=1, h=h,
                       init_state=init),
            oracle.Problem(Lx, Ly, cx, cy, d=2, periodic=periodic, J=J, U=0.0, model=1, h=h, init_state=init))


def _tables(init):
    t = oracle.neel_tables()
    return t if init == 1 else [t[0]]


def _cplx(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def _evolved_state(op, init, n, steps=6):
    _, rho = oracle.sample(op, _tables(init), seed=99, traj_offset=0, n_traj=n)
    return oracle.rk4(op, rho, 0.05, steps)


@pytest.mark.parametrize("shape", SHAPES)
def test_spin_sample_noise_bit_exact_codes(shape):
    gp, op = _probs(*shape)
    _say("spin sample_noise", shape)
    n = 6
    plan = cd.Plan(gp, n)
    assert plan.path == (5 if shape[2:4] == (2, 2) else 4)
    rho = plan.new_state()
    noise = torch.empty(n, plan.n_sites, plan.n_gen, dtype=torch.int8, device="cuda")
    plan.sample_noise(4321, 5, rho, noise=noise)
    torch.cuda.synchronize()
    codes, ref = oracle.sample(op, _tables(shape[5]), seed=4321, traj_offset=5, n_traj=n)
    assert np.array_equal(noise.cpu().numpy(), codes)
    assert np.abs(rho.cpu().numpy() - ref).max() < 1e-15


@pytest.mark.parametrize("shape", SHAPES)
def test_spin_fields_and_commutator(shape):
    gp, op = _probs(*shape)
    _say("spin fields/commutator", shape)
    n = 3
    rho = _evolved_state(op, shape[5], n)
    plan = cd.Plan(gp, n)
    r = _cplx(rho, torch.complex128)
    b = torch.empty(n, plan.n_sites, dtype=torch.complex128, device="cuda")
    phi = torch.empty_like(b)
    plan.gather_boundary_fields(r, b, phi)
    K = plan.new_state()
    ws = plan.new_workspace()
    plan.commutator(r, K, ws)
    torch.cuda.synchronize()
    bref, phiref = oracle.fields(op, rho)
    assert np.abs(b.cpu().numpy() - bref).max() < 1e-13
    assert np.abs(phi.cpu().numpy() - phiref).max() < 1e-13
    Kref = oracle.rhs(op, rho)
    assert np.abs(K.cpu().numpy() - Kref).max() < 1e-13 * max(np.abs(Kref).max(), 1.0)


@pytest.mark.parametrize("shape", SHAPES)
def test_spin_rk4_steps(shape):
    gp, op = _probs(*shape)
    _say("spin step_rk4", shape)
    n = 5
    rho = _evolved_state(op, shape[5], n, steps=2)
    plan = cd.Plan(gp, n)
    r = _cplx(rho, torch.complex128)
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.03, 9)
    torch.cuda.synchronize()
    assert np.abs(r.cpu().numpy() - oracle.rk4(op, rho, 0.03, 9)).max() < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_spin_observables(shape):
    gp, op = _probs(*shape)
    _say("spin observables", shape)
    n = 4
    rho = _evolved_state(op, shape[5], n)
    plan = cd.Plan(gp, n)
    r = _cplx(rho, torch.complex128)
    ws = plan.new_workspace()
    sums = torch.zeros(1, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(n, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(r, 0, sums, ws, per_traj=per)
    torch.cuda.synchronize()
    ref = oracle.observables(op, rho)
    got = per.cpu().numpy()
    assert np.all(np.abs(got[:, :13] - ref[:, :13]) < 1e-12 * np.maximum(1.0, np.abs(ref[:, :13])))
    assert np.all(got[:, 13:] < 1e-12) and np.all(ref[:, 13:] < 1e-12)
    assert np.allclose(sums.cpu().numpy()[0, :, 0], ref.sum(0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", [(4, 4, 2, 2, True, 1), (4, 1, 2, 1, False, 1), (6, 4, 1, 2, True, 0)])
@pytest.mark.parametrize("dtype", [1, 0])
def test_spin_quench(shape, dtype):
    gp, op = _probs(*shape, dtype=dtype)
    _say("spin quench", shape, "dtype", dtype)
    rec = [0, 10, 20, 40]
    n = 37   # a ragged last workgroup for every cluster shape
    sums, per = cd.run_quench(gp, n, seed=8, dt=0.025, record_steps=rec)
    ref = oracle.run(op, _tables(shape[5]), seed=8, traj_offset=0, n_traj=n, dt=0.025, n_steps=40,
                     record_steps=rec)["obs"]
    err = np.abs(per.numpy()[:, :, :12] - ref[:, :, :12]).max()
    _say("max err", err)
    assert err < (1e-10 if dtype == 1 else 2e-5)


def test_four_site_chain_against_exact_diagonalisation():
    """App. A: open four-site chain, two-site clusters, J = 1/8, h = 1, Neel
    start, 20000 trajectories.  The trajectory mean of M_z must agree with the
    method's exact expectation (oracle over all 256 noise configurations)
    within 5 standard errors, and stay within 0.02 of exact diagonalisation
    up to t = 4 (the method's own deviation there is below 0.011)."""
    Ns, Jc, h, dt = 4, 0.125, 1.0, 0.01
    gp, op = _probs(Ns, 1, 2, 1, False, 1, J=Jc, h=h)
    rec = list(range(0, 401, 50))
    n = 20000
    sums, _ = cd.run_quench(gp, n, seed=2024, dt=dt, record_steps=rec)
    mean, se = cd.estimates(sums, n)
    mz, mz_se = Ns * mean.numpy()[:, 0], Ns * se.numpy()[:, 0]
    codes = np.stack([np.array([[bits[2 * j], bits[2 * j + 1], 1 - j % 2] for j in range(Ns)], dtype=np.int8)
                      for bits in itertools.product((0, 1), repeat=2 * Ns)])
    rho = oracle.build_rho(op, oracle.neel_tables(), codes)
    Hm = ising_hamiltonian(Ns, [(0, 1), (1, 2), (2, 3)], Jc, h)
    r0 = spin_product_state([True, False, True, False])
    stag = sum(((-1) ** i) * spin_op(Ns, i, "z") for i in range(Ns))
    prev = 0
    for k, step in enumerate(rec):
        rho = oracle.rk4(op, rho, dt, step - prev)
        prev = step
        exact_method = Ns * oracle.observables(op, rho)[:, 0].mean()
        ed = np.real(np.trace(stag @ evolve(Hm, r0, dt * step)))
        _say(f"t={dt * step:.2f} gpu {mz[k]:+.4f} +- {mz_se[k]:.4f}  c-dtwa {exact_method:+.4f}  ed {ed:+.4f}")
        assert abs(mz[k] - exact_method) <= 5 * mz_se[k] + 1e-12
        assert abs(mz[k] - ed) < 0.02 + 5 * mz_se[k]


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


@pytest.mark.parametrize("lat", [(4, 4, True), (4, 6, False), (8, 4, True), (6, 6, False), (2, 2, False), (2, 4, False)])
@pytest.mark.parametrize("dtype", [1, 0])
def test_spin_fused_matches_oracle(lat, dtype):
    Lx, Ly, periodic = lat
    gp, op = _probs(Lx, Ly, 2, 2, periodic, 1, dtype=dtype)
    _say("spin fused vs oracle", lat, dtype)
    n = 3
    rho = _evolved_state(op, 1, n, steps=2)
    plan = cd.Plan(gp, n)
    assert plan.path == 5
    r = _cplx(rho, torch.complex128 if dtype == 1 else torch.complex64)
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.03, 12)
    assert plan.device_status(ws) == 0
    err = np.abs(r.cpu().numpy() - oracle.rk4(op, rho, 0.03, 12)).max()
    _say("max err", err)
    assert err < (1e-12 if dtype == 1 else 2e-5)


@pytest.mark.parametrize("dtype", [1, 0])
def test_spin_fused_rounds_equal_per_stage(dtype):
    """32x32 lattice, more trajectories than fit at once (several rounds),
    three calls (tags restart every call): the fused kernel against the
    per-stage spin kernels on the same noise."""
    gp, _ = _probs(32, 32, 2, 2, True, 1, dtype=dtype)
    n = cd.Plan(gp, 100000).resident + 3
    fused = cd.Plan(gp, n)
    per = _forced("spin", lambda: cd.Plan(gp, n))
    _say("spin fused rounds", dtype, "trajectories", n, "resident", fused.resident)
    assert fused.path == 5 and per.path == 4 and fused.resident < n
    a = fused.new_state()
    fused.sample_noise(77, 0, a)
    b = a.clone()
    wf, wp = fused.new_workspace(), per.new_workspace()
    for _ in range(3):
        fused.step_rk4(a, wf, 0.02, 4)
        per.step_rk4(b, wp, 0.02, 4)
    assert fused.device_status(wf) == 0
    err = (a - b).abs().max().item()
    _say("max |fused - per-stage|", err)
    assert err < (1e-12 if dtype == 1 else 2e-5)


def test_spin_fused_wait_timeout_is_reported():
    """A spin limit of 0 polls makes the fused spin kernel's neighbour waits
    time out: every wave still exits, the status word reports it and the
    affected clusters hold NaN; a normal plan afterwards is clean."""
    gp, _ = _probs(32, 32, 2, 2, True, 1)
    old = os.environ.get("CDTWA_SPIN_LIMIT")
    os.environ["CDTWA_SPIN_LIMIT"] = "0"
    try:
        plan = cd.Plan(gp, 3)
    finally:
        if old is None:
            os.environ.pop("CDTWA_SPIN_LIMIT", None)
        else:
            os.environ["CDTWA_SPIN_LIMIT"] = old
    assert plan.path == 5
    rho = plan.new_state()
    plan.sample_noise(9, 0, rho)
    ws = plan.new_workspace()
    plan.step_rk4(rho, ws, 0.01, 10)
    status = plan.device_status(ws)
    finite = bool(torch.isfinite(torch.view_as_real(rho)).all())
    _say("status", status, "finite", finite)
    assert status in (0, 1)
    assert (status == 1) == (not finite)
    normal = cd.Plan(gp, 3)
    r2 = normal.new_state()
    normal.sample_noise(9, 0, r2)
    w2 = normal.new_workspace()
    normal.step_rk4(r2, w2, 0.01, 10)
    assert normal.device_status(w2) == 0
    assert torch.isfinite(torch.view_as_real(r2)).all()


def test_spin_path_selection():
    gp, _ = _probs(4, 4, 2, 2, True, 1)
    assert cd.Plan(gp, 2).path == 5
    assert cd.Plan(_probs(4, 4, 2, 1, True, 1)[0], 2).path == 4      # the fused kernel is 2x2 only
    old = os.environ.get("CDTWA_PATH")
    try:
        os.environ["CDTWA_PATH"] = "plaq"
        with pytest.raises(cd.CdtwaError):
            cd.Plan(gp, 2)
        os.environ["CDTWA_PATH"] = "spin"
        assert cd.Plan(gp, 2).path == 4
        os.environ["CDTWA_PATH"] = "spinfused"
        assert cd.Plan(gp, 2).path == 5
        with pytest.raises(cd.CdtwaError):
            cd.Plan(cd.Problem(4, 4, 2, 2, d=3), 2)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old
    with pytest.raises(cd.CdtwaError):
        cd.Plan(cd.Problem(4, 4, 2, 2, d=3, model=1, h=1.0), 2)       # Ising needs d = 2
    with pytest.raises(cd.CdtwaError):
        cd.Plan(cd.Problem(4, 4, 2, 2, d=3, h=1.0), 2)                # h only for the Ising model
