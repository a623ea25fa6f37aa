"""Parity of the control-variate kernels (through the C ABI) with the oracle
in oracle/cv.py, and the statistical properties of the estimator.

Tolerances.  The device products take the same BF16 operands as the oracle
and accumulate in FP32 instead of FP64 (relative error ~1e-6 of the sum of
|terms|).  Where an FP32 pre-activation lands within that error of a BF16
rounding boundary the two sides round one activation to neighbouring BF16
values (one BF16 ulp, 2^-8 relative), which moves the downstream outputs by
about |W| * 2^-8 * |a|.  Such flips are rare (~1e-4 per activation), so the
bulk of the outputs agree to ~1e-5 of the output scale and every output to
2^-7 of it; gradients, sums over many rows, are compared in relative
Frobenius norm at 2e-3 (about the BF16 unit roundoff 2^-9).
Features, sampled features and noise codes are compared bit for bit; the
targets (FP64 arithmetic rounded once to FP32) to 1e-6 relative.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import cv as ocv

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")
from paper_2404_18594_amd import cv  # noqa: E402

TB = oracle.mott_tables(3)


def _say(*a):
    print(*a, flush=True)


def _params(seed):
    rng = np.random.default_rng(seed)
    parts = {}
    for name, shape in ocv.SHAPES:
        if len(shape) == 2:
            parts[name] = rng.uniform(-1, 1, size=shape) * np.sqrt(6.0 / shape[0])
        else:
            parts[name] = rng.uniform(-0.1, 0.1, size=shape)
    p32 = ocv.pack(parts).astype(np.float32)
    wq = np.concatenate([ocv.bf16_bits(p32[a:b]) for a, b in _weight_ranges()])
    return p32, wq


def _weight_ranges():
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in ocv.SHAPES])
    return [(offs[i], offs[i + 1]) for i in (0, 2, 4)]


def _mlp(p32, wq):
    m = cd.Mlp(seed=0)
    m.load(torch.from_numpy(p32).cuda(), torch.from_numpy(wq.view(np.int16)).cuda())
    return m


def _features(n, seed):
    """Inputs with the value set of real patch features (r^a values)."""
    rng = np.random.default_rng(seed)
    vals = np.array([-1.0, 0.0, 1.0, 2.0 / np.sqrt(3.0), -1.0 / np.sqrt(3.0)])
    return vals[rng.integers(0, len(vals), size=(n, ocv.NI))].astype(np.float32)


def _cmp_outputs(y, ref):
    scale = np.abs(ref).max()
    err = np.abs(y - ref)
    assert np.median(err) <= 1e-5 * scale, (np.median(err), scale)
    assert err.max() <= 2.0 ** -7 * scale, (err.max(), scale)


def test_mlp_init_properties():
    _say("mlp_init")
    m = cd.Mlp(seed=7)
    p = m.params.cpu().numpy()
    wq = m.wbf16.cpu().numpy().view(np.uint16)
    P = ocv.unpack(p)
    for name, fan_in, bound in (("W1", 128, np.sqrt(6 / 128)), ("W2", 256, np.sqrt(6 / 256)),
                                ("W3", 256, np.sqrt(3 / 256))):
        w = P[name]
        assert np.abs(w).max() <= bound and np.abs(w).max() > 0.95 * bound
        assert abs(w.mean()) < 0.02 * bound
        assert abs(w.var() - bound ** 2 / 3) < 0.05 * bound ** 2 / 3
    for name in ("b1", "b2", "b3"):
        assert np.all(P[name] == 0)
    ref = np.concatenate([ocv.bf16_bits(p[a:b]) for a, b in _weight_ranges()])
    assert np.array_equal(wq, ref)
    m2 = cd.Mlp(seed=7)
    assert torch.equal(m2.params, m.params)


@pytest.mark.parametrize("n", [16, 1000, 4096])
def test_mlp_forward_parity(n):
    _say("mlp_forward", n)
    p32, wq = _params(1)
    x = _features(n, 2)
    m = _mlp(p32, wq)
    y = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    ws = cd.Mlp.new_workspace(n)
    m.forward(torch.from_numpy(x).cuda(), y, ws)
    ref, _ = ocv.forward(p32.astype(np.float64), x, rounding=True)
    _cmp_outputs(y.cpu().numpy(), ref)


# 20480 rows: the column sums take chunks longer than their 64-row minimum
@pytest.mark.parametrize("n", [16, 1008, 4096, 20480])
def test_mlp_backward_parity(n):
    _say("mlp_backward", n)
    p32, wq = _params(3)
    x = _features(n, 4)
    rng = np.random.default_rng(5)
    t = rng.standard_normal((n, 64)).astype(np.float32)
    m = _mlp(p32, wq)
    y = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    ws = cd.Mlp.new_workspace(n)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.forward(torch.from_numpy(x).cuda(), y, ws)
    m.backward(y, torch.from_numpy(t).cuda(), ws, loss=loss)
    g = m.grad.cpu().numpy().astype(np.float64)
    yref, cache = ocv.forward(p32.astype(np.float64), x, rounding=True)
    gref = ocv.backward(cache, yref, t.astype(np.float64))
    assert abs(loss.item() - ocv.loss(yref, t)) <= 1e-4 * ocv.loss(yref, t)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in ocv.SHAPES])
    for i, (name, _) in enumerate(ocv.SHAPES):
        a, b = offs[i], offs[i + 1]
        rel = np.linalg.norm(g[a:b] - gref[a:b]) / np.linalg.norm(gref[a:b])
        _say(f"  {name}: rel {rel:.2e}")
        assert rel <= 2e-3, (name, rel)


def test_mlp_adam_parity():
    _say("mlp_adam")
    p32, wq = _params(6)
    rng = np.random.default_rng(7)
    m = _mlp(p32, wq)
    w = p32.astype(np.float64)
    mm = np.zeros_like(w)
    vv = np.zeros_like(w)
    lr = 1e-3
    for step in range(1, 4):
        g = (rng.standard_normal(w.size) * 10.0 ** rng.integers(-4, 1, w.size)).astype(np.float32)
        m.grad.copy_(torch.from_numpy(g))
        m.adam(lr)
        w, mm, vv = ocv.adam(w, g.astype(np.float64), mm, vv, lr, step)
    got = m.params.cpu().numpy().astype(np.float64)
    assert np.abs(got - w).max() <= 1e-6 * np.abs(w).max() + 1e-3 * lr
    wq2 = m.wbf16.cpu().numpy().view(np.uint16)
    ref = np.concatenate([ocv.bf16_bits(m.params.cpu().numpy()[a:b]) for a, b in _weight_ranges()])
    assert np.array_equal(wq2, ref)


@pytest.mark.parametrize("shape,periodic", [((8, 8), True), ((4, 6), False)])
def test_cv_features_bit_exact(shape, periodic):
    _say("cv_features", shape, periodic)
    n = 3
    plan = cd.Plan(cd.Problem(*shape, 2, 2, d=3, periodic=periodic), n)
    rho = plan.new_state()
    noise = torch.empty(n, plan.n_sites, plan.n_gen, dtype=torch.int8, device="cuda")
    plan.sample_noise(42, 5, rho, noise=noise)
    f = torch.empty(n * plan.n_clusters, 128, dtype=torch.float32, device="cuda")
    plan.cv_features(noise, f)
    op = oracle.Problem(*shape, 2, 2, d=3, periodic=periodic)
    codes, _ = oracle.sample(op, TB, seed=42, traj_offset=5, n_traj=n)
    assert np.array_equal(f.cpu().numpy(), ocv.features(op, TB, codes))


@pytest.mark.parametrize("shape,periodic,dtype", [((4, 4), True, 1), ((6, 4), False, 1), ((4, 4), True, 0)])
def test_cv_targets_parity(shape, periodic, dtype):
    _say("cv_targets", shape, periodic, dtype)
    n = 3
    op = oracle.Problem(*shape, 2, 2, d=3, periodic=periodic)
    _, rho = oracle.sample(op, TB, seed=9, traj_offset=0, n_traj=n)
    rho = oracle.rk4(op, rho, 0.05, 5)
    plan = cd.Plan(cd.Problem(*shape, 2, 2, d=3, periodic=periodic, dtype=dtype), n)
    cdt = torch.complex128 if dtype == 1 else torch.complex64
    r = torch.from_numpy(rho).to(cdt).cuda()
    ws = plan.new_workspace()
    t = torch.zeros(n * plan.n_clusters, 64, dtype=torch.float32, device="cuda")
    plan.cv_targets(r, 5, t, ws)
    got = t.cpu().numpy().reshape(n, plan.n_clusters, 64)
    ref = ocv.targets(op, rho)
    tol = 1e-6 if dtype == 1 else 2e-5
    assert np.abs(got[:, :, 5] - ref).max() <= tol * max(1.0, np.abs(ref).max())
    assert np.all(np.delete(got, 5, axis=2) == 0)


def test_cv_sample_features_bit_exact():
    _say("cv_sample_features")
    plan = cd.Plan(cd.Problem(4, 4, 2, 2, d=3), 1)
    f = torch.empty(300, 128, dtype=torch.float32, device="cuda")
    plan.cv_sample_features(0x123456789, 1000, f)
    ref = ocv.sample_patch_features(TB, 0x123456789, 1000, 300)
    assert np.array_equal(f.cpu().numpy(), ref)


def test_cv_traj_sums():
    _say("cv_traj_sums")
    n = 5
    plan = cd.Plan(cd.Problem(8, 4, 2, 2, d=3), n)
    rng = np.random.default_rng(8)
    y = rng.standard_normal((n * plan.n_clusters, 64)).astype(np.float32)
    g = torch.empty(n, 64, dtype=torch.float64, device="cuda")
    plan.cv_traj_sums(torch.from_numpy(y).cuda(), g)
    ref = y.astype(np.float64).reshape(n, plan.n_clusters, 64).sum(axis=1) / plan.n_sites
    assert np.abs(g.cpu().numpy() - ref).max() <= 1e-13


def test_cv_expectation_parity():
    """Two calls (the second adds into the same moments) across the chunk
    boundary of the device loop; the oracle runs the same patches."""
    _say("cv_expectation")
    p32, wq = _params(10)
    m = _mlp(p32, wq)
    plan = cd.Plan(cd.Problem(4, 4, 2, 2, d=3), 1)
    n = 33000
    fh = ocv.sample_patch_features(TB, 77, 0, n)
    mom = torch.zeros(64, 3, dtype=torch.float64, device="cuda")
    plan.cv_expectation(m, 77, n, mom)
    yref, _ = ocv.forward(p32.astype(np.float64), fh, rounding=True)
    got = mom.cpu().numpy()
    s = got[:, 0] + got[:, 1]
    scale = np.abs(yref).max()
    assert np.abs(s / n - yref.mean(axis=0)).max() <= 1e-5 * scale
    assert np.abs(got[:, 2] / n - (yref ** 2).mean(axis=0)).max() <= 1e-4 * scale ** 2
    plan.cv_expectation(m, 77, n, mom)
    got2 = mom.cpu().numpy()
    assert np.allclose(got2[:, 0] + got2[:, 1], 2 * s, rtol=1e-14, atol=1e-12)


def test_control_variate_unbiased_and_reduces_variance():
    """Train g on 256 trajectories of an 8x8 quench, evaluate on 512 fresh
    ones: the CV estimate agrees with the plain one within 4 combined
    standard errors at every time, and the variance drops at every time
    (most at t = 0, where O is a function of the patch noise alone)."""
    _say("control variate end to end")
    prob = cd.Problem(8, 8, 2, 2, d=3, periodic=True, J=1.0, U=5.0)
    rec = cv.record_schedule(40, 21)
    tr = cv.simulate(prob, 256, seed=1, traj_offset=0, dt=0.02, record_steps=rec, want_obs=False)
    mlp = cd.Mlp(seed=3)
    hist = cv.train(mlp, tr.features, tr.targets, epochs=60, batch=1024, lr=2e-3)
    _say("  loss", hist[0], hist[-1])
    assert hist[-1] < 0.5 * hist[0]
    ev = cv.simulate(prob, 512, seed=1, traj_offset=10_000, dt=0.02, record_steps=rec, want_targets=False)
    O, G = cv.observable_and_cv(ev, mlp)
    eg, varg = cv.expectation(ev.plan, mlp, seed=5, n_samples=200_000)
    est = cv.estimate(O, G, eg, varg, 200_000, ev.plan.n_clusters / ev.plan.n_sites)
    _say("  var ratio", np.round(est["var_ratio"], 3))
    z = np.abs(est["cv_mean"] - est["plain_mean"]) / np.sqrt(est["cv_se"] ** 2 + est["plain_se"] ** 2)
    assert np.all(z < 4), z
    assert est["var_ratio"][0] < 0.5
    assert np.all(est["var_ratio"] < 0.8)
