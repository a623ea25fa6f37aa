"""Pins of the control-variate oracle (oracle/cv.py).

* BF16 rounding: torch's own float32 -> bfloat16 conversion (nearest, ties
  to even) on random values and on exact ties.
* Backpropagation: central finite differences of the loss of the
  unrounded network, on a sample of every parameter block.
* Adam: the first step moves each weight by lr * g / (|g| + eps); with a
  constant gradient the bias-corrected moments equal g and g^2 at every step.
* Features: a roll-based extraction of the 4x4 patch from the lattice grid.
* Targets: summed over clusters and divided by Ns they equal
  (C^sp_(1,0) + C^sp_(0,1)) / 2 of the oracle's observable code (minimum-image
  ordered pairs, Sec. III definition of C^sp); for product states (t = 0)
  every pair term factorises.
* Sampler: outcome frequencies against the tomography probabilities.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import cv

TB = oracle.mott_tables(3)


def _params(rng, scale=1.0):
    P = {}
    for name, shape in cv.SHAPES:
        fan_in = shape[0] if len(shape) == 2 else 1
        P[name] = rng.uniform(-1, 1, size=shape) * scale * (np.sqrt(3.0 / fan_in) if len(shape) == 2 else 0.1)
    return cv.pack(P)


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e38, 1e-40]])
    # exact ties: 1 + 2^-8 (tie, even below), 1 + 3 * 2^-8 (tie, even above)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2 + 2.0 ** -7])
    x = np.concatenate([x, ties]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cv.bf16(x), ref)
    assert list(cv.bf16(ties[:2])) == [1.0, 1 + 2.0 ** -6]


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = _params(rng)
    x = rng.standard_normal((8, cv.NI))
    t = rng.standard_normal((8, cv.NO))
    y, cache = cv.forward(params, x, rounding=False)
    g = cv.backward(cache, y, t)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in cv.SHAPES])
    h = 1e-5
    for blk in range(len(cv.SHAPES)):
        idx = rng.integers(offs[blk], offs[blk + 1], size=12)
        for i in idx:
            pp, pm = params.copy(), params.copy()
            pp[i] += h
            pm[i] -= h
            fd = (cv.loss(cv.forward(pp, x, False)[0], t) - cv.loss(cv.forward(pm, x, False)[0], t)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (cv.SHAPES[blk][0], i, fd, g[i])


def test_rounded_network_within_bf16_bound():
    """Rounding every product operand to BF16 (relative error <= 2^-9) moves
    the outputs by a small multiple of 2^-9 of their scale."""
    rng = np.random.default_rng(2)
    params = _params(rng)
    x = rng.standard_normal((64, cv.NI))
    y0, _ = cv.forward(params, x, rounding=False)
    y1, _ = cv.forward(params, x, rounding=True)
    assert np.abs(y1 - y0).max() < 20 * 2.0 ** -9 * np.abs(y0).max()
    assert np.abs(y1 - y0).max() > 0


def test_adam_closed_forms():
    rng = np.random.default_rng(3)
    w = rng.standard_normal(1000)
    g = rng.standard_normal(1000)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-3
    w1, m1, v1 = cv.adam(w, g, m, v, lr, 1)
    assert np.allclose(w1 - w, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    # constant gradient: every step moves by the same amount
    ws, mm, vv = w.copy(), m, v
    for step in range(1, 30):
        w_next, mm, vv = cv.adam(ws, g, mm, vv, lr, step)
        assert np.allclose(w_next - ws, -lr * g / (np.abs(g) + 1e-8), rtol=1e-10, atol=1e-18)
        ws = w_next


@pytest.mark.parametrize("periodic", [True, False])
def test_features_roll_extraction(periodic):
    p = oracle.Problem(8, 4, 2, 2, J=1.0, U=5.0, periodic=periodic)
    codes, _ = oracle.sample(p, TB, seed=3, traj_offset=0, n_traj=2)
    f = cv.features(p, TB, codes).reshape(2, p.nc, 16, 8)
    for t in range(2):
        grid = np.zeros((p.Ly, p.Lx, 8))
        for j in range(p.Ns):
            grid[j // p.Lx, j % p.Lx] = [TB.val[a][codes[t, j, a]] for a in range(8)]
        if not periodic:   # pad with a ring of zeros, then roll inside the padded grid
            grid = np.pad(grid, ((1, 1), (1, 1), (0, 0)))
        for mu in range(p.nc):
            x0, y0 = (mu % (p.Lx // 2)) * 2, (mu // (p.Lx // 2)) * 2
            if periodic:
                patch = np.roll(np.roll(grid, -(y0 - 1), axis=0), -(x0 - 1), axis=1)[:4, :4]
            else:
                patch = np.roll(np.roll(grid, -y0, axis=0), -x0, axis=1)[:4, :4]
            assert np.array_equal(f[t, mu], patch.reshape(16, 8).astype(np.float32))


@pytest.mark.parametrize("shape,periodic", [((4, 4), True), ((8, 4), True), ((4, 6), False)])
def test_targets_sum_to_nearest_neighbour_csp(shape, periodic):
    p = oracle.Problem(*shape, 2, 2, J=1.0, U=5.0, periodic=periodic)
    res = oracle.run(p, TB, seed=4, traj_offset=0, n_traj=3, dt=0.02, n_steps=15, record_steps=[15],
                     want_rho=True)
    t = cv.targets(p, res["rho"])
    obs = oracle.observables(p, res["rho"])
    assert np.allclose(t.sum(axis=1) / p.Ns, 0.5 * (obs[:, 0] + obs[:, 1]), rtol=1e-12, atol=1e-14)


def test_targets_factorise_for_product_states():
    p = oracle.Problem(4, 4, 2, 2, J=1.0, U=5.0)
    _, rho = oracle.sample(p, TB, seed=8, traj_offset=0, n_traj=2)
    b, _ = oracle.fields(p, rho)
    t = cv.targets(p, rho)
    ref = np.zeros_like(t)
    sc, _, _, _ = oracle.maps(p)
    for i in range(p.Ns):
        x, y = i % 4, i // 4
        for j in (y * 4 + (x + 1) % 4, ((y + 1) % 4) * 4 + x):
            ref[:, sc[i]] += (np.conj(b[:, i]) * b[:, j]).real
    assert np.allclose(t, ref, rtol=1e-12, atol=1e-14)


def test_patch_sampler_frequencies():
    n = 400
    f = cv.sample_patch_features(TB, seed=11, first=0, n=n).reshape(n * 16, 8)
    for a in range(8):
        for o in range(TB.n_out[a]):
            k = np.sum(np.isclose(f[:, a], TB.val[a][o]))
            pr = TB.prob[a][o]
            sd = np.sqrt(n * 16 * pr * (1 - pr)) + 1e-9
            assert abs(k - n * 16 * pr) < 5 * sd, (a, o, k, n * 16 * pr)
    # chunks compose: patches 100..149 drawn alone equal rows 100..149
    g = cv.sample_patch_features(TB, seed=11, first=100, n=50)
    assert np.array_equal(g, f.reshape(n, 128)[100:150])
    # the C loop and the Python statement of the counter layout agree, also
    # past 2^32 patches (upper counter word) and with a 64-bit seed
    for seed, first in ((11, 0), (0xDEADBEEF12345678, (1 << 32) - 3)):
        assert np.array_equal(cv.sample_patch_features(TB, seed, first, 6),
                              cv.sample_patch_features_py(TB, seed, first, 6))
