"""Pins of the oracle's time-dependent couplings (RK4 with J(t), U(t) -- or
J(t), h(t) for the Ising model -- sampled at every half step; stage 1 at t,
stages 2 and 3 at t + dt/2, stage 4 at t + dt).  The paper ramps the
couplings in its Fig. 2 protocol (Sec. III); the schedule is the caller's.

* A constant schedule equals the constant-coupling RK4 exactly.
* One cluster covering an open lattice (no mean-field coupling): RK4 of the
  Mott product matrix equals the exact time-dependent von Neumann evolution
  (independent full-space Hamiltonians, SciPy's DOP853 at 1e-12) with a
  global error that falls 16-fold when dt halves -- a stage evaluated at the
  wrong time would leave a first- or second-order error.
* 1x1 clusters: the oracle follows the single-site SU(3) dTWA in the r^a
  variables (tests/exact.py) with the same time-dependent couplings,
  integrated by DOP853.
* Ising: one two-site cluster with J(t), h(t) against the exact evolution.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from exact import (DtwaR, bh_hamiltonian, ising_hamiltonian, product_fock, single_site_op, spin_op,
                   spin_product_state)


def Jt(t):
    return 1.0 + 0.5 * np.sin(3.0 * t)


def Ut(t):
    return 6.0 - 4.0 * t + np.cos(t)


def _half(f, dt, n):
    return np.array([f(0.5 * dt * k) for k in range(2 * n + 1)])


def _exact(Hc1, Hc2, rho0, T):
    D = rho0.shape[0]

    def rhs(t, y):
        r = y.reshape(D, D)
        H = Jt(t) * Hc1 + Ut(t) * Hc2
        return (-1j * (H @ r - r @ H)).ravel()
    sol = solve_ivp(rhs, (0, T), rho0.ravel().astype(complex), method="DOP853", rtol=1e-12, atol=1e-13)
    return sol.y[:, -1].reshape(D, D)


def test_constant_schedule_equals_rk4():
    p = oracle.Problem(4, 4, 2, 2, d=3, periodic=True, J=0.8, U=5.0)
    _, rho = oracle.sample(p, oracle.mott_tables(3), seed=3, traj_offset=0, n_traj=2)
    a = oracle.rk4(p, rho, 0.02, 5)
    b = oracle.rk4_schedule(p, rho, 0.02, 5, np.full(11, 0.8), np.full(11, 5.0))
    assert np.array_equal(a, b)


def test_single_cluster_follows_time_dependent_exact_evolution():
    Lx, Ly, d, T = 2, 1, 3, 0.6
    p = oracle.Problem(Lx, Ly, 2, 1, d=d, periodic=False, J=1.0, U=1.0)
    Hc1 = bh_hamiltonian(2, [(0, 1)], d, 1.0, 0.0)
    Hc2 = bh_hamiltonian(2, [(0, 1)], d, 0.0, 1.0)
    rho0 = product_fock(2, d, [1, 1])
    exact = _exact(Hc1, Hc2, rho0, T)
    errs = []
    for n in (30, 60):
        dt = T / n
        out = oracle.rk4_schedule(p, rho0[None, None], dt, n, _half(Jt, dt, n), _half(Ut, dt, n))[0, 0]
        errs.append(np.abs(out - exact).max())
    assert errs[1] < 1e-6
    assert 12 < errs[0] / errs[1] < 20, errs


def test_one_site_clusters_follow_time_dependent_dtwa():
    Lx, Ly, dt, n = 3, 3, 0.0025, 160
    p = oracle.Problem(Lx, Ly, 1, 1, d=3, periodic=True, J=1.0, U=1.0)
    tb = oracle.mott_tables(3)
    codes, rho = oracle.sample(p, tb, seed=17, traj_offset=0, n_traj=3)
    got = oracle.observables(p, oracle.rk4_schedule(p, rho, dt, n, _half(Jt, dt, n), _half(Ut, dt, n)))
    model = DtwaR(Lx, Ly, True, 3, 1.0, 1.0, tb.T)
    eta_u1 = model.eta_U.copy()

    def rhs(t, y):
        model.J = Jt(t)
        model.eta_U = Ut(t) * eta_u1
        return model.rhs(y.reshape(p.Ns, 8)).ravel()
    for t in range(3):
        r0 = np.array([[tb.val[a, codes[t, j, a]] for a in range(8)] for j in range(p.Ns)])
        sol = solve_ivp(rhs, (0, dt * n), r0.ravel(), method="DOP853", rtol=1e-12, atol=1e-12)
        ref = model.observables(sol.y[:, -1].reshape(p.Ns, 8))
        assert np.allclose(got[t, :11], ref, atol=1e-6, rtol=0)   # RK4 error at dt = 0.0025: ~2e-7


def test_ising_cluster_follows_time_dependent_exact_evolution():
    T, n = 0.8, 400
    dt = T / n
    p = oracle.Problem(2, 1, 2, 1, d=2, periodic=False, J=1.0, U=0.0, model=1, h=1.0, init_state=1)
    Hc1 = ising_hamiltonian(2, [(0, 1)], 1.0, 0.0)
    Hc2 = ising_hamiltonian(2, [(0, 1)], 0.0, 1.0)
    rho0 = spin_product_state([True, False])
    exact = _exact(Hc1, Hc2, rho0, T)
    out = oracle.rk4_schedule(p, rho0[None, None], dt, n, _half(Jt, dt, n), _half(Ut, dt, n))[0, 0]
    assert np.abs(out - exact).max() < 5e-7   # h(t) ~ 7: RK4 error ~1e-7 at dt = 0.002
