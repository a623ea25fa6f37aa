"""Pins of the oracle's dynamics against exact results.

* A single cluster that covers a whole open lattice has no mean-field
  coupling, so the equation of motion is the exact von Neumann equation and
  the method becomes exact as the cluster grows to the system (arXiv:2404.18594,
  Sec. III, last paragraphs; App. B.1, E[A_tot] = rho(0)).  The oracle's RK4
  must then reproduce exact diagonalisation up to the O(dt^4) RK4 error, and be
  linear in the initial matrix.
* For 1x1 clusters the method is the single-site SU(d) dTWA; written in the
  variables r^a with structure constants it must agree with the oracle to
  rounding (RK4 commutes with the affine map A <-> r).
Both pins run at d = 3 (the paper's SU(3) case, App. B.1) and at d = 4 (the
generalised Gell-Mann basis of SU(4), D = 256 for 2x2 clusters).
"""
import itertools

import numpy as np
import pytest

import oracle
from exact import DtwaR, bh_hamiltonian, evolve, product_fock, single_site_op


def _positions(cx, cy):
    # local index l = x*cy + y
    return [(l // cy, l % cy) for l in range(cx * cy)]


def _bonds(pos):
    return [(i, j) for i in range(len(pos)) for j in range(i + 1, len(pos))
            if abs(pos[i][0] - pos[j][0]) + abs(pos[i][1] - pos[j][1]) == 1]


# (d, cluster shape, initial occupations).  At d = 4 the occupations start
# from 3 and 2 on some sites as well as 1, so that the sqrt(3) entries of a
# and a^+ and the interaction 3U of n = 3 enter from the first step, and the
# 2x2 cluster covers every Kronecker stride of D = 256.
SINGLE_CLUSTER_CASES = [
    (3, (2, 1), (1, 1)), (3, (1, 2), (1, 1)), (3, (2, 2), (1, 1, 1, 1)),
    (4, (2, 1), (3, 1)), (4, (1, 2), (2, 3)), (4, (2, 2), (1, 3, 2, 0)), (4, (2, 2), (1, 1, 1, 1)),
]


@pytest.mark.parametrize("d,shape,occ", SINGLE_CLUSTER_CASES)
def test_single_cluster_rk4_equals_exact_diagonalisation(d, shape, occ):
    cx, cy = shape
    J, U, T = 1.0, 5.0, 0.5
    p = oracle.Problem(cx, cy, cx, cy, d=d, periodic=False, J=J, U=U)
    pos = _positions(cx, cy)
    H = bh_hamiltonian(len(pos), _bonds(pos), d, J, U)
    rho0 = product_fock(len(pos), d, list(occ))
    exact = evolve(H, rho0, T)
    # the exact evolution must leave the initial state far enough for the
    # comparison to see every matrix element of H that it reaches
    assert np.abs(exact - rho0).max() > 0.05
    errs = []
    # the d = 4 starts reach energies up to ~20 J (n = 3 costs 3U): finer steps
    for n in ((50, 100) if d == 3 else (100, 200)):
        rho = oracle.rk4(p, rho0[None, None], T / n, n)[0, 0]
        errs.append(np.abs(rho - exact).max())
    assert errs[1] < 5e-7
    assert 10 < errs[0] / errs[1] < 22          # fourth-order convergence


def test_single_cluster_d4_reaches_triple_occupation():
    """The d = 4 single-cluster pin above is only a pin of the n = 3 matrix
    elements if the dynamics populates n = 3: with a site started at n = 3 it
    must also leave it (through the sqrt(3) of a), and with the Mott start two
    hops must fill a site to n = 3."""
    J, U, T = 1.0, 5.0, 0.5
    for occ, site in (((3, 1), 0), ((1, 1, 1, 1), 1)):
        n_sites = len(occ)
        cx, cy = (2, 1) if n_sites == 2 else (2, 2)
        p = oracle.Problem(cx, cy, cx, cy, d=4, periodic=False, J=J, U=U)
        rho0 = product_fock(n_sites, 4, list(occ))
        rho = oracle.rk4(p, rho0[None, None], T / 100, 100)[0, 0]
        P3 = np.diag([1.0 if s[site] == 3 else 0.0 for s in itertools.product(range(4), repeat=n_sites)])
        p3 = float(np.real(np.trace(P3 @ rho)))
        if occ[site] == 3:
            assert p3 < 0.98
        else:
            assert p3 > 1e-4


def test_single_cluster_is_linear_in_the_initial_matrix():
    p = oracle.Problem(2, 2, 2, 2, periodic=False)
    tb = oracle.mott_tables(3)
    _, rho = oracle.sample(p, tb, seed=3, traj_offset=0, n_traj=3)
    w = np.array([0.2, 0.5, 0.3])
    mix = np.einsum("n,nij->ij", w, rho[:, 0])[None, None]
    ev_mix = oracle.rk4(p, mix, 0.01, 30)[0, 0]
    ev = oracle.rk4(p, rho, 0.01, 30)[:, 0]
    assert np.abs(ev_mix - np.einsum("n,nij->ij", w, ev)).max() < 1e-12


def _site_configs(tb):
    choices = [[(n, tb.prob[a, n]) for n in range(tb.n_out[a]) if tb.prob[a, n] > 1e-12] for a in range(tb.n_gen)]
    for combo in itertools.product(*choices):
        yield np.array([c[0] for c in combo], dtype=np.int8), float(np.prod([c[1] for c in combo]))


@pytest.mark.parametrize("shape", [(2, 1), (1, 2)])
def test_enumerated_noise_average_equals_exact(shape):
    """Average of the whole pipeline (sampling rule -> cluster product -> RK4 ->
    observables) over the complete discrete noise distribution equals the exact
    expectation values of the two-site lattice."""
    cx, cy = shape
    J, U, T, n = 1.0, 5.0, 0.4, 80
    p = oracle.Problem(cx, cy, cx, cy, periodic=False, J=J, U=U)
    tb = oracle.mott_tables(3)
    cfg = list(_site_configs(tb))
    codes, weights = [], []
    for c0, c1 in itertools.product(cfg, cfg):
        codes.append(np.stack([c0[0], c1[0]]))
        weights.append(c0[1] * c1[1])
    codes = np.array(codes)
    weights = np.array(weights)
    rho = oracle.build_rho(p, tb, codes)
    rho_t = oracle.rk4(p, rho, T / n, n)
    obs = oracle.observables(p, rho_t)
    mean = weights @ obs
    pos = _positions(cx, cy)
    H = bh_hamiltonian(2, _bonds(pos), 3, J, U)
    ex = evolve(H, product_fock(2, 3, [1, 1]), T)
    g01 = np.real(np.trace(single_site_op(2, 3, 0, "adag") @ single_site_op(2, 3, 1, "a") @ ex))
    nn = np.real(np.trace(single_site_op(2, 3, 0, "n") @ single_site_op(2, 3, 1, "n") @ ex))
    cls = 0 if cx == 2 else 1                     # (1,0) along x, (0,1) along y
    # C^sp = (1/Ns) sum over the two ordered pairs = Re <a0^+ a1>
    assert abs(mean[cls] - g01) < 1e-8
    assert abs(mean[5 + cls] - nn) < 1e-8
    assert abs(mean[10] - 1.0) < 1e-12


@pytest.mark.parametrize("d", [3, 4])
@pytest.mark.parametrize("lat", [(4, 4, True), (3, 3, True), (3, 2, False)])
def test_one_site_clusters_equal_dtwa_in_r_variables(lat, d):
    Lx, Ly, periodic = lat
    J, U, dt, n = 1.0, 5.0, 0.02, 25
    p = oracle.Problem(Lx, Ly, 1, 1, d=d, periodic=periodic, J=J, U=U)
    tb = oracle.mott_tables(d)
    res = oracle.run(p, tb, seed=11, traj_offset=0, n_traj=6, dt=dt, n_steps=n, record_steps=[0, n],
                     want_codes=True)
    model = DtwaR(Lx, Ly, periodic, d, J, U, tb.T)
    for t in range(6):
        r0 = np.array([[tb.val[a, res["codes"][t, j, a]] for a in range(tb.n_gen)] for j in range(p.Ns)])
        for k, steps in enumerate((0, n)):
            ref = model.observables(model.rk4(r0, dt, steps))
            assert np.allclose(res["obs"][t, k, :11], ref, atol=1e-11, rtol=0)
