"""Physics sanity of the method (parity unpinned: the method is an
approximation).  On a 3x2 open lattice the C-dTWA with 1x1 and 1x2 clusters
must agree with exact diagonalisation at short times within the Monte-Carlo
error (arXiv:2404.18594, Sec. III: the cluster method captures the early-time
correlation growth)."""
import numpy as np
import pytest

import oracle
from exact import bh_hamiltonian, evolve, product_fock, single_site_op


@pytest.mark.parametrize("shape", [(1, 1), (1, 2)])
def test_short_time_correlations_match_exact(shape):
    Lx, Ly, J, U = 3, 2, 1.0, 5.0
    sites = [(x, y) for y in range(Ly) for x in range(Lx)]
    bonds = [(i, j) for i in range(6) for j in range(i + 1, 6)
             if abs(sites[i][0] - sites[j][0]) + abs(sites[i][1] - sites[j][1]) == 1]
    H = bh_hamiltonian(6, bonds, 3, J, U)
    ad = [single_site_op(6, 3, j, "adag") for j in range(6)]
    a = [single_site_op(6, 3, j, "a") for j in range(6)]
    p = oracle.Problem(Lx, Ly, *shape, periodic=False, J=J, U=U)
    n = 4000
    res = oracle.run(p, oracle.mott_tables(3), seed=1, traj_offset=0, n_traj=n, dt=0.01,
                     n_steps=10, record_steps=[5, 10])
    m = res["obs"].mean(0)
    se = res["obs"].std(0) / np.sqrt(n)
    for k, t in enumerate((0.05, 0.1)):
        ex = evolve(H, product_fock(6, 3, [1] * 6), t)
        for cls, (dx, dy) in enumerate(((1, 0), (0, 1))):
            c = sum(np.real(np.trace(ad[i] @ a[j] @ ex)) for i in range(6) for j in range(6)
                    if i != j and abs(sites[i][0] - sites[j][0]) == dx and abs(sites[i][1] - sites[j][1]) == dy) / 6
            assert abs(m[k, cls] - c) < 4 * se[k, cls] + 1e-3
