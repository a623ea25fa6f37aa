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
Besides these random-input checks, `test_mlp_elementwise_on_exact_grid`
compares every output and every gradient entry on inputs for which BF16
operands and FP32 accumulation are provably exact: bit for bit, or within the
rigorous summation bound where a sum may round.
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


# ---------------------------------------------------------------------------
# Element-by-element parity on dyadic-grid inputs.  Features in {-1, 0, 1},
# weights k/16 (|k| <= 4), biases odd multiples of 1/32, 1/1024 (layers 1
# and 2, so no pre-activation can be exactly 0 and the ReLU masks agree) and
# k/16 (layer 3), targets y_ref - j/8 (|j| <= 3) and a power-of-two row count
# (so dy = 2 (y - t) / (64 n) is exact).  Every operand of every product is
# then a BF16 value with few significant bits, every product is exact in
# FP32, and a sum of such products is exact in FP32 in ANY order whenever
# the sum of the magnitudes of its terms stays below 2^24 units of the
# coarsest common power of two of the terms.  That is proved on the CPU for
# each sum before the comparison (`_exact`).  Exact sums are compared bit for
# bit; a sum that may round (the weight gradients over 32768 rows) is
# compared entry by entry against the rigorous bound of floating-point
# summation, |fl(sum) - sum| <= (K + 1) u sum |terms| with K the number of
# terms and u = 2^-24 (the +1 is the final FP32 store), with every operand
# of it still bit-identical on both sides.
# ---------------------------------------------------------------------------
U32 = 2.0 ** -24


def _lsb_exp(v):
    """Exponent of the lowest set bit over the nonzero entries of v."""
    v = np.asarray(v, dtype=np.float64).ravel()
    v = v[v != 0]
    if v.size == 0:
        return 0
    m, e = np.frexp(np.abs(v))
    ints = (m * 2.0 ** 53).astype(np.int64)
    return int((e - 53 + np.log2(ints & -ints).astype(np.int64)).min())


def _exact(A, B, bias=None):
    """(exact, sum of |terms|) of the product A B (+ bias) summed in FP32 in
    any order."""
    u = _lsb_exp(A) + _lsb_exp(B)
    S = np.abs(A) @ np.abs(B)
    if bias is not None:
        u = min(u, _lsb_exp(bias))
        S = S + np.abs(bias)
    return bool(S.max() < 2.0 ** (24 + u)), S


def _colsum_exact(X):
    S = np.abs(X).sum(axis=0)
    return bool(S.max() < 2.0 ** (24 + _lsb_exp(X))), S


def _grid_params(seed):
    rng = np.random.default_rng(seed)
    parts = {"W1": rng.integers(-4, 5, size=(128, 256)) / 16.0,
             "b1": (2 * rng.integers(-4, 4, size=256) + 1) / 32.0,
             "W2": rng.integers(-4, 5, size=(256, 256)) / 16.0,
             "b2": (2 * rng.integers(-4, 4, size=256) + 1) / 1024.0,
             "W3": rng.integers(-4, 5, size=(256, 64)) / 16.0,
             "b3": rng.integers(-8, 9, size=64) / 16.0}
    p = ocv.pack(parts)
    p32 = p.astype(np.float32)
    assert np.array_equal(p32.astype(np.float64), p)
    wq = np.concatenate([ocv.bf16_bits(p32[a:b]) for a, b in _weight_ranges()])
    assert np.array_equal(ocv.bf16(p32), p)           # every parameter is a BF16 value
    return p, p32, wq, parts


def _check_block(name, got, ref, exact, S, K):
    err = np.abs(got.astype(np.float64) - ref)
    if exact:
        bad = np.count_nonzero(err)
        _say(f"  {name}: exact sums, {bad} entries differ")
        assert bad == 0, (name, err.max())
    else:
        bound = (K + 1) * U32 * S
        _say(f"  {name}: sums may round, max err / bound {float((err / np.maximum(bound, 1e-300)).max()):.3f}, "
             f"{np.count_nonzero(err)} of {err.size} entries not bit-equal")
        assert np.all(err <= bound), (name, float((err - bound).max()))


@pytest.mark.parametrize("n", [64, 1024, 32768])
def test_mlp_elementwise_on_exact_grid(n):
    _say("mlp elementwise", n)
    p, p32, wq, P = _grid_params(11)
    rng = np.random.default_rng(12)
    x = rng.integers(-1, 2, size=(n, 128)).astype(np.float64)
    yref, c = ocv.forward(p, x, rounding=True)
    # premise: the forward sums are exact and no pre-activation is 0
    for A, B, b in ((c["x0"], P["W1"], P["b1"]), (c["a1"], P["W2"], P["b2"]), (c["a2"], P["W3"], P["b3"])):
        assert _exact(A, B, b)[0]
    assert np.all(c["z1"] != 0) and np.all(c["z2"] != 0)
    m = _mlp(p32, wq)
    y = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    ws = cd.Mlp.new_workspace(n)
    m.forward(torch.from_numpy(x.astype(np.float32)).cuda(), y, ws)
    yg = y.cpu().numpy()
    assert np.array_equal(yg.astype(np.float64), yref), np.abs(yg - yref).max()
    # backward: targets one coarse step away from the exact outputs
    e = rng.integers(-3, 4, size=yref.shape) / 8.0
    t = yref - e
    assert np.array_equal(t.astype(np.float32).astype(np.float64), t)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.backward(y, torch.from_numpy(t.astype(np.float32)).cuda(), ws, loss=loss)
    gref = ocv.backward(c, yref, t)
    G, R = ocv.unpack(m.grad.cpu().numpy()), ocv.unpack(gref)
    assert loss.item() == ocv.loss(yref, t)
    # the operands of the backward products, as the oracle forms them
    dyq = ocv.bf16(2.0 * e / (n * 64))
    assert np.array_equal(dyq, 2.0 * e / (n * 64))
    ex_da2, _ = _exact(dyq, P["W3"].T)
    dz2 = (dyq @ P["W3"].T) * (c["z2"] > 0)
    dz2q = ocv.bf16(dz2)
    ex_da1, _ = _exact(dz2q, P["W2"].T)
    dz1 = (dz2q @ P["W2"].T) * (c["z1"] > 0)
    dz1q = ocv.bf16(dz1)
    # da2 and da1 must be exact so that both sides round the same dz2, dz1
    assert ex_da2 and ex_da1
    for name, A, B in (("W3", c["a2"].T, dyq), ("W2", c["a1"].T, dz2q), ("W1", c["x0"].T, dz1q)):
        ex, S = _exact(A, B)
        _check_block(name, G[name], R[name], ex, S, n)
    for name, X in (("b3", 2.0 * e / (n * 64)), ("b2", dz2), ("b1", dz1)):
        ex, S = _colsum_exact(X)
        _check_block(name, G[name], R[name], ex, S, n)


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
