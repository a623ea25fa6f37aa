"""Pins of the fixed-N sector exact dynamics (oracle/ed.py), the reference for
the method's physics error on the 4x4 periodic quench of Sec. III.

* Against an independent full-space ED (tests/exact.py: every occupation
  tuple of every particle number, dense eigen-decomposition, observables from
  single-site operator matrices) on an open 3x2 lattice.
* Sector dimension: for d = 3 and N = Ns it is the central trinomial
  coefficient sum_k Ns! / (k! k! (Ns - 2k)!).
* Invariants: norm, particle number and energy are conserved; the
  translation-invariant shortcut for periodic lattices equals the full sum
  over ordered pairs.
"""
from math import factorial

import numpy as np
import pytest

from exact import bh_hamiltonian, evolve, product_fock, single_site_op
from oracle import ed


def _full_space_observables(Lx, Ly, d, J, U, t):
    Ns = Lx * Ly
    bonds = ed.lattice_bonds(Lx, Ly, False)
    H = bh_hamiltonian(Ns, bonds, d, J, U)
    rho = evolve(H, product_fock(Ns, d, [1] * Ns), t)
    a = [single_site_op(Ns, d, j, "a") for j in range(Ns)]
    ad = [single_site_op(Ns, d, j, "adag") for j in range(Ns)]
    n = [single_site_op(Ns, d, j, "n") for j in range(Ns)]
    out = np.zeros(12)
    for c, lst in enumerate(ed.class_pairs(Lx, Ly, False)):
        for (i, j) in lst:
            out[c] += np.real(np.trace(ad[i] @ a[j] @ rho))
            out[5 + c] += np.real(np.trace(n[i] @ n[j] @ rho))
    out[:10] /= Ns
    out[10] = sum(np.real(np.trace(n[j] @ rho)) for j in range(Ns)) / Ns
    out[11] = np.real(np.trace(H @ rho)) / Ns
    return out


@pytest.mark.parametrize("t", [0.0, 0.15, 0.6])
def test_sector_matches_full_space_ed(t):
    Lx, Ly, d, J, U = 3, 2, 3, 1.0, 4.0
    s = ed.Sector(Lx, Ly, d, Lx * Ly, False, J, U)
    psi = s.evolve(s.fock([1] * s.Ns), [0.0, t])[-1] if t > 0 else s.fock([1] * s.Ns)
    got = s.observables(psi)
    ref = _full_space_observables(Lx, Ly, d, J, U, t)
    assert np.abs(got - ref).max() < 1e-10


@pytest.mark.parametrize("Ns", [4, 6, 9])
def test_sector_dimension_is_central_trinomial(Ns):
    L = {4: (2, 2), 6: (3, 2), 9: (3, 3)}[Ns]
    s = ed.Sector(L[0], L[1], 3, Ns, False, 1.0, 1.0)
    trinomial = sum(factorial(Ns) // (factorial(k) ** 2 * factorial(Ns - 2 * k)) for k in range(Ns // 2 + 1))
    assert s.dim == trinomial
    assert (np.diff(s.codes) > 0).all()


def test_periodic_invariants_and_translation_shortcut():
    s = ed.Sector(3, 3, 3, 9, True, 1.0, 19.6)
    assert len(s.bonds) == 18
    times = np.linspace(0.0, 0.5, 6)
    psi = s.evolve(s.fock([1] * 9), times)
    e0 = None
    for p in psi:
        assert abs(np.vdot(p, p).real - 1.0) < 1e-12
        full = s.observables(p)
        assert abs(full[10] - 1.0) < 1e-12
        e0 = full[11] if e0 is None else e0
        assert abs(full[11] - e0) < 1e-10
        assert abs(full[11]) < 1e-10        # <Mott| H |Mott> = 0: no double occupancy, no diagonal hop
    s2 = ed.Sector(3, 3, 3, 9, True, 1.0, 19.6)
    for p in psi:
        assert np.abs(s2.observables(p, translation_invariant=True) - s.observables(p)).max() < 1e-12
