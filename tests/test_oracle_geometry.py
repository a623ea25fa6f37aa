"""Pins of the oracle's cluster geometry against the explicit 2x2 cluster
Hamiltonian of arXiv:2404.18594, App. B.1 (Gamma^intra and the eight legs of
Phi^inter), and of its neighbour tables against their definitions."""
import numpy as np
import pytest

import oracle
from conftest import read_golden


def test_intra_cluster_bonds_match_paper():
    gold = {tuple(sorted(int(x) for x in r)) for r in read_golden("cluster2x2_intra_bonds.txt")}
    _, _, _, bonds = oracle.maps(oracle.Problem(4, 4, 2, 2))
    got = {tuple(sorted(int(x) + 1 for x in b)) for b in bonds}
    assert got == gold


@pytest.mark.parametrize("L", [4, 6, 8])
def test_inter_cluster_legs_match_paper(L):
    p = oracle.Problem(L, L, 2, 2)
    sc, sl, nb, _ = oracle.maps(p)
    ncx = L // 2
    gold = sorted((int(r[0]), int(r[1]), int(r[2]), int(r[3])) for r in read_golden("cluster2x2_legs.txt"))
    for mu in range(p.nc):
        mx, my = mu % ncx, mu // ncx
        legs = []
        for j in np.where(sc == mu)[0]:
            for k in range(4):
                n = nb[j, k]
                if n < 0 or sc[n] == mu:
                    continue
                nx, ny = sc[n] % ncx, sc[n] // ncx
                dmx = (nx - mx + ncx // 2) % ncx - ncx // 2 if ncx > 2 else (nx - mx) % ncx
                dmy = (ny - my + ncx // 2) % ncx - ncx // 2 if ncx > 2 else (ny - my) % ncx
                legs.append((int(sl[j]) + 1, int(sl[n]) + 1, dmx, dmy))
        if ncx > 2:
            assert sorted(legs) == gold
        else:
            # with two clusters per direction the offsets +1 and -1 coincide
            assert sorted((a, b) for a, b, _, _ in legs) == sorted((a, b) for a, b, _, _ in gold)


@pytest.mark.parametrize("shape", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_neighbour_tables(shape):
    cx, cy = shape
    for periodic, L in ((True, 4), (False, 4), (True, 6)):
        p = oracle.Problem(L, L, cx, cy, periodic=periodic)
        sc, sl, nb, bonds = oracle.maps(p)
        for j in range(p.Ns):
            x, y = j % L, j // L
            assert sc[j] == (y // cy) * (L // cx) + x // cx
            assert sl[j] == (x % cx) * cy + (y % cy)
            for k, (dx, dy) in enumerate(((1, 0), (-1, 0), (0, 1), (0, -1))):
                xx, yy = x + dx, y + dy
                if periodic:
                    assert nb[j, k] == (yy % L) * L + (xx % L)
                elif 0 <= xx < L and 0 <= yy < L:
                    assert nb[j, k] == yy * L + xx
                else:
                    assert nb[j, k] == -1
        assert len(bonds) == {1: 0, 2: 1, 4: 4}[cx * cy]


def test_rejects_self_coupled_periodic_lattices():
    for p in (oracle.Problem(2, 4, 2, 2), oracle.Problem(2, 2, 1, 1), oracle.Problem(3, 4, 2, 2)):
        with pytest.raises(ValueError):
            oracle.geometry(p)
