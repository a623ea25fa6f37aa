"""Invariant and metamorphic pins of the oracle (arXiv:2404.18594).

* Each cluster matrix evolves by a commutator with a Hermitian generator
  (Sec. II Eq. (cluster_mf)): trace and Hermiticity are kept exactly by the
  flow, Tr A^2 and the spectrum are kept by the flow (RK4 error only).
* The hops between clusters cancel pairwise in the total particle number, so
  N_MF is a linear invariant that RK4 keeps to rounding; the mean-field energy
  is quadratic and drifts at the RK4 order dt^4.
* The number of noises and the initial state do not depend on the clustering
  (Sec. II, the total number of random variables is independent of the cluster
  choice); with J = 0 there is no coupling at all, so every clustering gives
  the same trajectory.
* Lattice translations, the x<->y reflection and a global U(1) phase are
  symmetries of the Bose-Hubbard Hamiltonian and of the Mott state.
"""
import numpy as np
import pytest

import oracle

TB = oracle.mott_tables(3)


def test_per_trajectory_invariants():
    p = oracle.Problem(4, 4, 2, 2, J=1.0, U=5.0)
    res = oracle.run(p, TB, seed=5, traj_offset=0, n_traj=4, dt=0.01, n_steps=100, record_steps=[0, 50, 100])
    obs = res["obs"]
    assert np.all(obs[:, :, 13] < 1e-12)                # |Tr A - 1|
    assert np.all(obs[:, :, 14] < 1e-12)                # |A - A^+|
    assert np.allclose(obs[:, :, 10], 1.0, atol=1e-13)   # N_MF / Ns
    assert np.allclose(obs[:, 0, 12], 81.0, atol=1e-12)   # Tr A^2 at t = 0
    # Tr A^2 is kept by the exact flow; RK4 damps it at high order in dt
    loss = []
    for n in (50, 100):
        r = oracle.run(p, TB, seed=5, traj_offset=0, n_traj=2, dt=0.5 / n, n_steps=n, record_steps=[n])
        loss.append(np.abs(r["obs"][:, 0, 12] - 81.0).max())
    assert loss[1] < 2e-4 and loss[0] / loss[1] > 16


def test_energy_drift_is_fourth_order():
    p = oracle.Problem(4, 4, 2, 2, J=1.0, U=5.0)
    T = 0.5
    drift = []
    for n in (25, 50):
        res = oracle.run(p, TB, seed=9, traj_offset=0, n_traj=2, dt=T / n, n_steps=n, record_steps=[0, n])
        drift.append(np.abs(res["obs"][:, 1, 11] - res["obs"][:, 0, 11]).max())
    assert drift[1] < 1e-6
    assert 8 < drift[0] / drift[1] < 40


@pytest.mark.parametrize("J", [1.0, 0.0])
def test_clustering_independence(J):
    """Same noise, four clusterings: identical observables at t = 0 and
    identical d<a_j>/dt at t = 0; with J = 0 identical trajectories."""
    L = 4
    res, rates = {}, {}
    for shape in ((1, 1), (2, 1), (1, 2), (2, 2)):
        p = oracle.Problem(L, L, *shape, J=J, U=5.0)
        r = oracle.run(p, TB, seed=21, traj_offset=0, n_traj=3, dt=0.02, n_steps=20, record_steps=[0, 20],
                       want_codes=True)
        res[shape] = r
        _, rho0 = oracle.sample(p, TB, seed=21, traj_offset=0, n_traj=3)
        K = oracle.rhs(p, rho0)
        rates[shape] = oracle.fields(p, K)[0]             # Tr(a_j K) = d<a_j>/dt
    ref = res[(1, 1)]
    for shape, r in res.items():
        assert np.array_equal(r["codes"], ref["codes"])
        assert np.allclose(r["obs"][:, 0, :12], ref["obs"][:, 0, :12], atol=1e-12)
        assert np.allclose(rates[shape], rates[(1, 1)], atol=1e-12)
        if J == 0.0:
            # the exact flows agree; the RK4 polynomial of a sum of commuting
            # single-site terms differs from the product of single-site RK4
            # polynomials at O(dt^5) per step, so agreement is to RK4 order
            assert np.allclose(r["obs"][:, 1, :12], ref["obs"][:, 1, :12], atol=1e-5)
    if J == 0.0:
        diffs = []
        for dt, n in ((0.02, 20), (0.01, 40)):
            o = [oracle.run(oracle.Problem(L, L, *s, J=0.0, U=5.0), TB, seed=21, traj_offset=0, n_traj=3, dt=dt,
                            n_steps=n, record_steps=[n])["obs"][:, 0, :12] for s in ((1, 1), (2, 2))]
            diffs.append(np.abs(o[0] - o[1]).max())
        assert diffs[0] / diffs[1] > 12


def _evolve_obs(p, rho, n=40, dt=0.01):
    return oracle.observables(p, oracle.rk4(p, rho, dt, n))


def test_translation_by_one_cluster():
    p = oracle.Problem(6, 4, 2, 2)
    _, rho = oracle.sample(p, TB, seed=2, traj_offset=0, n_traj=2)
    ncx, ncy = 3, 2
    perm = [((mu // ncx) * ncx + (mu % ncx + 1) % ncx) for mu in range(p.nc)]
    shifted = rho[:, perm]
    a = _evolve_obs(p, rho)
    b = _evolve_obs(p, shifted)
    assert np.allclose(a, b, atol=1e-11)
    # fields are translated with the state
    ba, _ = oracle.fields(p, oracle.rk4(p, rho, 0.01, 10))
    bb, _ = oracle.fields(p, oracle.rk4(p, shifted, 0.01, 10))
    for j in range(p.Ns):
        x, y = j % 6, j // 6
        assert np.allclose(bb[:, j], ba[:, y * 6 + (x + 2) % 6], atol=1e-12)


def test_reflection_x_y():
    p = oracle.Problem(4, 4, 2, 2)
    _, rho = oracle.sample(p, TB, seed=4, traj_offset=0, n_traj=2)
    # swapping x and y swaps local sites 1 and 2 (local index x*2 + y) and
    # transposes the cluster grid
    D = 81
    P = np.zeros((D, D))
    for q in range(D):
        n = [(q // 27) % 3, (q // 9) % 3, (q // 3) % 3, q % 3]
        m = [n[0], n[2], n[1], n[3]]
        P[m[0] * 27 + m[1] * 9 + m[2] * 3 + m[3], q] = 1.0
    refl = np.empty_like(rho)
    for mu in range(4):
        mx, my = mu % 2, mu // 2
        refl[:, mx * 2 + my] = P @ rho[:, mu] @ P.T
    a = _evolve_obs(p, rho)
    b = _evolve_obs(p, refl)
    swap = [1, 0, 2, 4, 3, 6, 5, 7, 9, 8, 10, 11, 12, 13, 14]
    assert np.allclose(a[:, swap], b, atol=1e-11)


def test_global_phase_rotation():
    p = oracle.Problem(4, 4, 2, 2)
    _, rho = oracle.sample(p, TB, seed=6, traj_offset=0, n_traj=2)
    theta = 0.7
    v = np.exp(1j * theta * np.arange(3))
    V = v
    for _ in range(3):
        V = np.kron(V, v)
    rot = V[None, None, :, None] * rho * V.conj()[None, None, None, :]
    a = _evolve_obs(p, rho)
    b = _evolve_obs(p, rot)
    assert np.allclose(a, b, atol=1e-11)
