"""Pins of the oracle's transverse-field Ising model (App. A, Eq. (Hising)):
H = J sum_<ij> s^z_i s^z_j + h sum_i s^x_i, spin 1/2, Neel initial state with
s^x and s^y drawn as +-1 with probability 1/2 and s^z fixed.

* The cluster Hamiltonian is compared with one built element by element.
* One cluster covering an open chain has no mean-field coupling; the average
  over all 2^(2 Ns) equally likely noise configurations of the initial matrix
  is the initial density matrix, and the evolution is linear, so that average
  must equal exact diagonalisation up to the RK4 error.
* With 1x1 clusters every trajectory is a set of classical Pauli vectors in
  the field B_j = (h, 0, J sum_k s^z_k): the oracle's matrix equation must
  follow the Bloch equations integrated independently (this pins the sign and
  size of the inter-cluster coupling, kappa = J/2 with B = B^+ = s^z).
* Closed forms: J = 0 rotates every spin about x at angular frequency 2h;
  h = 0 conserves s^z.  Energy is conserved by every trajectory.
* The four-site chain with two-site clusters, J = 1/8, h = 1 (App. A,
  figure of M_z): the exact C-dTWA average (all 256 noise configurations)
  stays close to exact diagonalisation.
"""
import itertools

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from exact import bloch_rhs, evolve, ising_hamiltonian, spin_op, spin_product_state


def _chain(Ns, cx, J, h, periodic=False):
    return oracle.Problem(Ns, 1, cx, 1, d=2, periodic=periodic, J=J, U=0.0, model=1, h=h, init_state=1)


def _all_codes(Ns):
    """Every noise configuration of a Neel chain: generators (s^x, s^y, s^z)
    with outcome index 0 -> -1 and 1 -> +1; s^z fixed by the sublattice."""
    out = []
    for bits in itertools.product((0, 1), repeat=2 * Ns):
        c = np.zeros((Ns, 3), dtype=np.int8)
        for j in range(Ns):
            c[j, 0], c[j, 1] = bits[2 * j], bits[2 * j + 1]
            c[j, 2] = 1 if j % 2 == 0 else 0
        out.append(c)
    return np.stack(out)


def test_cluster_hamiltonian_matches_elementwise():
    J, h = 0.3, 0.7
    p = _chain(2, 2, J, h)
    _, _, N, H0 = oracle.operators(p)
    assert np.allclose(H0, ising_hamiltonian(2, [(0, 1)], J, h), atol=1e-15)
    for l in range(2):
        assert np.allclose(N[l], spin_op(2, l, "x"), atol=1e-15)


def test_sampling_follows_the_neel_tables():
    p = _chain(4, 2, 0.125, 1.0)
    codes, rho = oracle.sample(p, oracle.neel_tables(), seed=11, traj_offset=0, n_traj=4000)
    # s^z fixed: +1 on even sites, -1 on odd sites
    assert (codes[:, 0::2, 2] == 1).all() and (codes[:, 1::2, 2] == 0).all()
    # s^x and s^y fair coins, independent across generators and sites
    f = codes[:, :, :2].reshape(len(codes), -1).astype(float)
    assert np.abs(f.mean(0) - 0.5).max() < 0.035
    c = np.corrcoef(f.T)
    assert np.abs(c - np.eye(len(c))).max() < 0.08
    # each A_j is I/2 + (1/2) sum_a r^a s^a: trace 1, Tr(A_j^2) = (1 + 3)/2
    obs = oracle.observables(p, rho)
    assert np.allclose(obs[:, 12], 4.0) and np.allclose(obs[:, 0], 1.0)


@pytest.mark.parametrize("J,h", [(0.125, 1.0), (1.0, 0.6)])
def test_single_cluster_average_equals_exact_diagonalisation(J, h):
    Ns, dt, n_steps = 2, 0.005, 300
    p = _chain(Ns, 2, J, h)
    codes = _all_codes(Ns)
    rho = oracle.rk4(p, oracle.build_rho(p, oracle.neel_tables(), codes), dt, n_steps)
    obs = oracle.observables(p, rho).mean(0)
    H = ising_hamiltonian(Ns, [(0, 1)], J, h)
    r = evolve(H, spin_product_state([True, False]), dt * n_steps)
    sz = [np.real(np.trace(spin_op(Ns, i, "z") @ r)) for i in range(Ns)]
    sx = [np.real(np.trace(spin_op(Ns, i, "x") @ r)) for i in range(Ns)]
    sy = [np.real(np.trace(spin_op(Ns, i, "y") @ r)) for i in range(Ns)]
    zz = np.real(np.trace(spin_op(Ns, 0, "z") @ spin_op(Ns, 1, "z") @ r))
    assert obs[0] == pytest.approx((sz[0] - sz[1]) / Ns, abs=1e-8)
    assert obs[1] == pytest.approx(np.mean(sz), abs=1e-8)
    assert obs[2] == pytest.approx(np.mean(sx), abs=1e-8)
    assert obs[3] == pytest.approx(np.mean(sy), abs=1e-8)
    assert obs[5] == pytest.approx(2 * zz / Ns, abs=1e-8)
    assert obs[11] == pytest.approx(np.real(np.trace(H @ r)) / Ns, abs=1e-8)


@pytest.mark.parametrize("periodic", [False, True])
def test_single_site_clusters_follow_bloch_equations(periodic):
    Ns, J, h, dt, n_steps = 4, 0.8, 1.0, 0.005, 200
    p = _chain(Ns, 1, J, h, periodic)
    tb = oracle.neel_tables()
    if periodic:
        p = oracle.Problem(3, 4, 1, 1, d=2, periodic=True, J=J, U=0.0, model=1, h=h, init_state=1)
        Ns = 12
    codes, rho = oracle.sample(p, tb, seed=5, traj_offset=0, n_traj=6)
    out = oracle.observables(p, oracle.rk4(p, rho, dt, n_steps))
    _, _, nb, _ = oracle.maps(p)
    nbrs = [[int(k) for k in row if k >= 0] for row in nb]
    T = dt * n_steps
    for t in range(len(codes)):
        s0 = np.array([[tb[0].val[a][codes[t, j, a]] for a in range(3)] for j in range(Ns)], dtype=float)
        sol = solve_ivp(lambda _, y: bloch_rhs(y.reshape(Ns, 3), nbrs, J, h).ravel(), (0, T), s0.ravel(),
                        method="DOP853", rtol=1e-12, atol=1e-12)
        s = sol.y[:, -1].reshape(Ns, 3)
        stag = np.array([(-1) ** ((j % p.Lx) + (j // p.Lx)) for j in range(Ns)])
        # RK4 at dt = 0.005 with fields up to 4J: global error ~1e-8
        assert out[t, 0] == pytest.approx((stag * s[:, 2]).mean(), abs=1e-7)
        assert out[t, 1:4] == pytest.approx(s[:, [2, 0, 1]].mean(0), abs=1e-7)
        # energy of the classical spins, h sum s^x + J sum_bonds s^z s^z, at T
        # and at t = 0 (conserved by the Bloch equations)
        def energy(v):
            return h * v[:, 0].sum() + 0.5 * J * sum(v[i, 2] * v[k, 2] for i in range(Ns) for k in nbrs[i])
        assert out[t, 11] == pytest.approx(energy(s) / Ns, abs=1e-7)
        assert out[t, 11] == pytest.approx(energy(s0) / Ns, abs=1e-7)


def test_closed_forms():
    Ns, dt, n_steps = 4, 0.01, 100
    T = dt * n_steps
    tb = oracle.neel_tables()
    # J = 0: rotation about x at 2h, per trajectory
    h = 0.9
    p = _chain(Ns, 2, 0.0, h)
    codes, rho = oracle.sample(p, tb, seed=2, traj_offset=0, n_traj=8)
    out = oracle.observables(p, oracle.rk4(p, rho, dt, n_steps))
    c, s = np.cos(2 * h * T), np.sin(2 * h * T)
    for t in range(len(codes)):
        v = np.array([[tb[0].val[a][codes[t, j, a]] for a in range(3)] for j in range(Ns)], dtype=float)
        # ds^y/dt = -2h s^z, ds^z/dt = 2h s^y
        sy = v[:, 1] * c - v[:, 2] * s
        sz = v[:, 2] * c + v[:, 1] * s
        assert out[t, 1] == pytest.approx(sz.mean(), abs=1e-8)
        assert out[t, 3] == pytest.approx(sy.mean(), abs=1e-8)
        assert out[t, 2] == pytest.approx(v[:, 0].mean(), abs=1e-12)
    # h = 0: s^z conserved on every site
    p = _chain(Ns, 2, 0.7, 0.0)
    codes, rho = oracle.sample(p, tb, seed=3, traj_offset=0, n_traj=8)
    out = oracle.observables(p, oracle.rk4(p, rho, dt, n_steps))
    assert np.allclose(out[:, 0], 1.0, atol=1e-12) and np.allclose(out[:, 1], 0.0, atol=1e-12)


def test_four_site_chain_tracks_exact_diagonalisation():
    Ns, J, h, dt = 4, 0.125, 1.0, 0.01
    record = [0, 50, 100, 150, 200, 300, 400]
    p = _chain(Ns, 2, J, h)
    codes = _all_codes(Ns)
    rho = oracle.build_rho(p, oracle.neel_tables(), codes)
    H = ising_hamiltonian(Ns, [(0, 1), (1, 2), (2, 3)], J, h)
    r0 = spin_product_state([True, False, True, False])
    stag = sum(((-1) ** i) * spin_op(Ns, i, "z") for i in range(Ns))
    prev = 0
    for step in record:
        rho = oracle.rk4(p, rho, dt, step - prev)
        prev = step
        mz = Ns * oracle.observables(p, rho)[:, 0].mean()
        ed = np.real(np.trace(stag @ evolve(H, r0, dt * step)))
        assert abs(mz - ed) < 0.06, (step, mz, ed)
