"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, entry
point by entry point and for whole quenches, on identical seeded inputs.

Tolerances.  FP64: the GPU and the oracle differ only in summation order and
fused multiply-adds, i.e. a few ulp per operation; errors then grow with the
dynamics (the mean-field flow is chaotic), so single stages are compared at
1e-12 relative and trajectories of O(1)/J duration at 1e-10 absolute on O(1)
observables.  FP32: the state is rounded to 2^-24 relative at every stage;
over the short runs here the observables stay within 2e-5 absolute.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


SHAPES = [
    # (Lx, Ly, cx, cy, d, periodic)
    (4, 4, 2, 2, 3, True),
    (6, 4, 2, 2, 3, True),
    (4, 4, 2, 2, 3, False),
    (4, 6, 1, 1, 3, True),
    (4, 4, 2, 1, 3, True),
    (4, 4, 1, 2, 3, False),
    (4, 4, 2, 2, 2, True),
    (4, 4, 2, 1, 4, True),
    (3, 3, 1, 1, 4, True),
    (4, 4, 2, 2, 4, True),     # D = 256: the cluster matrix exceeds the LDS (one launch per stage)
    (4, 6, 2, 2, 4, False),
    (6, 6, 2, 2, 4, True),     # 9 clusters, odd trajectory count: some clusters straddle two XCD ranges
    (2, 2, 2, 2, 4, False),    # one cluster, open: every boundary field vanishes
]


def _probs(Lx, Ly, cx, cy, d, periodic, dtype=1, J=1.0, U=5.0):
    return (cd.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=J, U=U, dtype=dtype),
            oracle.Problem(Lx, Ly, cx, cy, d=d, periodic=periodic, J=J, U=U))


def _cplx(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("shape", SHAPES)
def test_sample_noise_bit_exact_codes(shape):
    gp, op = _probs(*shape)
    _say("sample_noise", shape)
    n = 5
    plan = cd.Plan(gp, n)
    rho = plan.new_state()
    noise = torch.empty(n, plan.n_sites, plan.n_gen, dtype=torch.int8, device="cuda")
    plan.sample_noise(1234, 77, rho, noise=noise)
    torch.cuda.synchronize()
    codes, ref = oracle.sample(op, oracle.mott_tables(shape[4]), seed=1234, traj_offset=77, n_traj=n)
    assert np.array_equal(noise.cpu().numpy(), codes)
    assert np.abs(rho.cpu().numpy() - ref).max() < 1e-14


def _evolved_state(op, d, n, steps=6):
    _, rho = oracle.sample(op, oracle.mott_tables(d), seed=99, traj_offset=0, n_traj=n)
    return oracle.rk4(op, rho, 0.05, steps)


@pytest.mark.parametrize("shape", SHAPES)
def test_fields_and_commutator(shape):
    gp, op = _probs(*shape)
    _say("fields/commutator", shape)
    n = 3
    rho = _evolved_state(op, shape[4], n)
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
    scale = np.abs(Kref).max()
    assert np.abs(K.cpu().numpy() - Kref).max() < 1e-13 * max(scale, 1.0)


@pytest.mark.parametrize("shape", SHAPES)
def test_rk4_steps(shape):
    gp, op = _probs(*shape)
    _say("step_rk4", shape)
    n = 3
    rho = _evolved_state(op, shape[4], n, steps=2)
    plan = cd.Plan(gp, n)
    r = _cplx(rho, torch.complex128)
    ws = plan.new_workspace()
    plan.step_rk4(r, ws, 0.03, 7)
    torch.cuda.synchronize()
    ref = oracle.rk4(op, rho, 0.03, 7)
    assert np.abs(r.cpu().numpy() - ref).max() < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_observables(shape):
    gp, op = _probs(*shape)
    _say("observables", shape)
    n = 4
    rho = _evolved_state(op, shape[4], n)
    plan = cd.Plan(gp, n)
    r = _cplx(rho, torch.complex128)
    ws = plan.new_workspace()
    sums = torch.zeros(2, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(n, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(r, 1, sums, ws, per_traj=per)
    plan.accumulate_observables(r, 1, sums, ws, per_traj=per)
    torch.cuda.synchronize()
    ref = oracle.observables(op, rho)
    got = per.cpu().numpy()
    # purity sums D^2 terms: relative bound
    assert np.all(np.abs(got[:, :13] - ref[:, :13]) < 1e-12 * np.maximum(1.0, np.abs(ref[:, :13])))
    assert np.all(got[:, 13:] < 1e-12) and np.all(ref[:, 13:] < 1e-12)
    s = sums.cpu().numpy()
    assert np.all(s[0] == 0)
    assert np.allclose(s[1, :, 0] + s[1, :, 1], 2 * ref.sum(0), rtol=1e-13, atol=1e-13)
    assert np.allclose(s[1, :, 2], 2 * (ref ** 2).sum(0), rtol=1e-12, atol=1e-12)


NON_HERMITIAN_CASES = [
    # (Lx, Ly, cx, cy, d, model, n): the persistent D = 81 kernel on a count
    # of clusters that is not a multiple of its grid, the four-wave kernel
    # (D = 9), the one-wave kernel (D = 3), D = 256 and the spin model
    pytest.param(6, 6, 2, 2, 3, 0, 31, id="6x6_2x2_d3_D81"),
    pytest.param(6, 4, 2, 1, 3, 0, 7, id="6x4_2x1_d3_D9"),
    pytest.param(5, 3, 1, 1, 3, 0, 5, id="5x3_1x1_d3_D3"),
    pytest.param(4, 4, 2, 2, 4, 0, 2, id="4x4_2x2_d4_D256"),
    pytest.param(4, 4, 2, 2, 2, 1, 5, id="4x4_2x2_spin_D16"),
]


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
@pytest.mark.parametrize("Lx,Ly,cx,cy,d,model,n", NON_HERMITIAN_CASES)
def test_observables_non_hermitian(Lx, Ly, cx, cy, d, model, n, dtype):
    """Every observable against the oracle to 1e-12 on random non-Hermitian
    cluster matrices, where Tr rho^2 = sum Y_pq Y_qp, the complex trace
    deviation and the Hermiticity deviation differ from their Hermitian
    forms.  The FP32 case gives the oracle the same FP32 values."""
    _say("observables non-Hermitian", (Lx, Ly, cx, cy, d, model, n), "dtype", dtype)
    kw = dict(d=d, periodic=True, J=1.0, U=5.0 if model == 0 else 0.0)
    if model == 1:
        kw.update(model=1, h=1.0)
    gp = cd.Problem(Lx, Ly, cx, cy, dtype=dtype, **kw)
    op = oracle.Problem(Lx, Ly, cx, cy, **kw)
    plan = cd.Plan(gp, n)
    D = plan.D
    rng = np.random.default_rng(1000 * D + n)
    shape = (n, plan.n_clusters, D, D)
    rho = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / D
    if dtype == cd.F32:
        rho = rho.astype(np.complex64).astype(np.complex128)
    r = torch.from_numpy(rho.astype(np.complex128 if dtype == cd.F64 else np.complex64)).cuda()
    ws = plan.new_workspace()
    sums = torch.zeros(1, cd.NOBS, 3, dtype=torch.float64, device="cuda")
    per = torch.zeros(n, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.accumulate_observables(r, 0, sums, ws, per_traj=per)
    torch.cuda.synchronize()
    ref = oracle.observables(op, rho)
    got = per.cpu().numpy()
    assert ref[:, 14].min() > 1e-3                      # far from Hermitian
    bad = np.abs(got - ref) > 1e-12 * np.maximum(1.0, np.abs(ref))
    assert not bad.any(), [(int(t), int(k), got[t, k], ref[t, k]) for t, k in zip(*np.nonzero(bad))][:8]


def test_config_quench_4x4_2x2_fp64():
    """4x4 periodic lattice, four 2x2 clusters (D = 81), U/J = 5, dt = 0.05 to
    T = 1/J (20 steps), 32 trajectories from seed 0: per-trajectory
    observables at all 21 times."""
    gp, op = _probs(4, 4, 2, 2, 3, True)
    _say("quench 4x4 2x2 fp64")
    rec = list(range(21))
    sums, per = cd.run_quench(gp, 32, seed=0, dt=0.05, record_steps=rec)
    ref = oracle.run(op, oracle.mott_tables(3), seed=0, traj_offset=0, n_traj=32, dt=0.05, n_steps=20,
                     record_steps=rec)["obs"]
    err = np.abs(per.numpy()[:, :, :13] - ref[:, :, :13]).max()
    _say("max err", err)
    assert err < 1e-10
    mean, se = cd.estimates(sums, 32)
    assert np.allclose(mean.numpy()[:, :13], ref.mean(0)[:, :13], atol=1e-11)


@pytest.mark.parametrize("shape", [(4, 4, 2, 2, 3, True), (4, 6, 1, 1, 3, True), (4, 4, 2, 1, 3, False),
                                   (4, 4, 2, 2, 4, True)])
def test_quench_fp32(shape):
    gp, op = _probs(*shape, dtype=0)
    _say("quench fp32", shape)
    rec = [0, 5, 10]
    # d = 4: the interaction reaches 3U per site and dt = 0.05 leaves the RK4
    # stability region (the oracle diverges too); 0.02 is inside it
    dt = 0.05 if shape[4] < 4 else 0.02
    sums, per = cd.run_quench(gp, 7, seed=3, dt=dt, record_steps=rec)
    ref = oracle.run(op, oracle.mott_tables(shape[4]), seed=3, traj_offset=0, n_traj=7, dt=dt, n_steps=10,
                     record_steps=rec)["obs"]
    err = np.abs(per.numpy()[:, :, :12] - ref[:, :, :12]).max()
    _say("max err", err)
    assert err < 2e-5


def test_batched_driver_matches_single_batch():
    gp, _ = _probs(6, 4, 2, 2, 3, True)
    _say("batching")
    a, pa = cd.run_quench(gp, 9, seed=5, dt=0.05, record_steps=[0, 3])
    b, pb = cd.run_quench(gp, 9, seed=5, dt=0.05, record_steps=[0, 3], batch=4)
    assert torch.equal(pa, pb)
    assert torch.allclose(a[..., 0] + a[..., 1], b[..., 0] + b[..., 1], rtol=1e-14, atol=1e-14)
