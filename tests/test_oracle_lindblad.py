"""Pins of the oracle's open-system extension: local Lindblad channels on
every cluster matrix, L_j = sqrt(gdeph) n_j (dephasing) and sqrt(gloss) a_j
(loss), K += L Y L^+ - (L^+ L Y + Y L^+ L)/2 (the paper names the extension
to the Lindblad master equation; the channels are the standard local ones).

* One cluster covering an open lattice: RK4 of the initial matrix equals
  exact Lindblad evolution, exp(L t) of an independently built Liouvillian
  superoperator (row-major vectorisation, vec(A X B) = (A kron B^T) vec X),
  with a 16-fold error drop when dt halves.
* J = 0, loss only (any U, any dephasing): d<n>/dt = -gloss <n> exactly in
  the truncated space (a^+ n a = n (n - 1)), so the density of every
  trajectory decays as exp(-gloss t).
* J = 0, dephasing only: every entry of a cluster matrix evolves as
  Y_pq exp(-i (E_p - E_q) t - gdeph/2 sum_l (n_l(p) - n_l(q))^2 t).
* Trace and Hermiticity are kept on a periodic lattice with mean fields.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
from exact import bh_hamiltonian, product_fock, single_site_op


def _liouvillian(H, jumps):
    D = H.shape[0]
    I = np.eye(D)
    Lv = -1j * (np.kron(H, I) - np.kron(I, H.T))
    for L in jumps:
        LdL = L.conj().T @ L
        Lv += np.kron(L, L.conj()) - 0.5 * np.kron(LdL, I) - 0.5 * np.kron(I, LdL.T)
    return Lv


@pytest.mark.parametrize("gd,gl", [(0.7, 0.0), (0.0, 0.9), (0.4, 0.6)])
def test_single_cluster_equals_exact_lindblad(gd, gl):
    d, J, U, T = 3, 1.0, 4.0, 0.5
    p = oracle.Problem(2, 1, 2, 1, d=d, periodic=False, J=J, U=U, gdeph=gd, gloss=gl)
    H = bh_hamiltonian(2, [(0, 1)], d, J, U)
    jumps = [np.sqrt(gd) * single_site_op(2, d, j, "n") for j in range(2)] + \
            [np.sqrt(gl) * single_site_op(2, d, j, "a") for j in range(2)]
    rho0 = product_fock(2, d, [1, 2])
    exact = (expm(_liouvillian(H, jumps) * T) @ rho0.ravel()).reshape(9, 9)
    errs = []
    for n in (25, 50):
        out = oracle.rk4(p, rho0[None, None], T / n, n)[0, 0]
        errs.append(np.abs(out - exact).max())
    assert errs[1] < 1e-6
    assert 12 < errs[0] / errs[1] < 20, errs


def test_loss_decays_density_exactly():
    gl, T, n = 0.8, 0.6, 60
    p = oracle.Problem(4, 4, 2, 2, d=3, periodic=True, J=0.0, U=5.0, gdeph=0.3, gloss=gl)
    _, rho = oracle.sample(p, oracle.mott_tables(3), seed=4, traj_offset=0, n_traj=2)
    obs = oracle.observables(p, oracle.rk4(p, rho, T / n, n))
    assert np.allclose(obs[:, 10], np.exp(-gl * T), atol=1e-9)


def test_dephasing_closed_form():
    gd, U, T, n = 0.9, 3.0, 0.5, 100
    p = oracle.Problem(4, 4, 2, 1, d=3, periodic=True, J=0.0, U=U, gdeph=gd)
    _, rho = oracle.sample(p, oracle.mott_tables(3), seed=6, traj_offset=0, n_traj=2)
    out = oracle.rk4(p, rho, T / n, n)
    occ = np.array([[q // 3, q % 3] for q in range(9)])        # local 0 most significant
    E = U * 0.5 * (occ * (occ - 1)).sum(axis=1)
    dn2 = ((occ[:, None, :] - occ[None, :, :]) ** 2).sum(axis=2)
    factor = np.exp(-1j * (E[:, None] - E[None, :]) * T - 0.5 * gd * dn2 * T)
    assert np.abs(out - rho * factor).max() < 1e-8


def test_trace_and_hermiticity_with_mean_fields():
    p = oracle.Problem(4, 4, 2, 2, d=3, periodic=True, J=1.0, U=5.0, gdeph=0.5, gloss=0.5)
    _, rho = oracle.sample(p, oracle.mott_tables(3), seed=9, traj_offset=0, n_traj=2)
    obs = oracle.observables(p, oracle.rk4(p, rho, 0.02, 10))
    assert obs[:, 13].max() < 1e-12 and obs[:, 14].max() < 1e-12
    assert (obs[:, 10] < 1.0).all()       # particles leave
