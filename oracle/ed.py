"""Exact quantum dynamics of the truncated Bose-Hubbard model in a fixed
particle-number sector -- TEST INFRASTRUCTURE ONLY.

This is not the C-dTWA: it is the exact evolution |psi(t)> = exp(-iHt)|psi0>
that the method approximates (Sec. III, the 4x4 periodic sudden quench from
the unit-filling Mott state to U/J = 19.6 and its comparison with numerically
exact results).  It measures the method's physics error; it is never a parity
reference for the GPU path.  Only the tests, the scripts that write the stored
expected values under tests/golden/, and the benchmark's CPU-baseline leg may
use it.  It shares nothing with the GPU library.

Model (Sec. III Eq. (H_bose)): H = -J sum_<ij> (a_i^+ a_j + h.c.)
+ U/2 sum_i n_i (n_i - 1) on an Lx x Ly lattice, site j = y*Lx + x, with
occupations truncated to 0..d-1 as in the method (d = n_max + 1).

Basis: all occupation tuples with sum N, encoded as the base-d integer
sum_j n_j d^j, in ascending code order.  H is assembled bond by bond as a
sparse matrix; the state is propagated with SciPy's expm_multiply
(truncated Taylor series with scaling, Al-Mohy and Higham 2011).

Observables use the oracle's layout (slots 0..11): for each displacement
class c of (1,0),(0,1),(1,1),(2,0),(0,2) (minimum image if periodic),
slot c = (1/Ns) sum over ordered pairs (i,j) in class c of Re <a_i^+ a_j>,
slot 5+c the same sum of <n_i n_j>, slot 10 = (1/Ns) sum_j <n_j>,
slot 11 = <H>/Ns.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import expm_multiply

CLASSES = ((1, 0), (0, 1), (1, 1), (2, 0), (0, 2))


def _min_image(dd: int, L: int, periodic: bool) -> int:
    if not periodic:
        return abs(dd)
    m = dd % L
    return min(m, L - m)


def lattice_bonds(Lx: int, Ly: int, periodic: bool):
    """Nearest-neighbour bonds (i, j), each once (+x and +y neighbours)."""
    bonds = set()
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            for dx, dy in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if periodic:
                    xx %= Lx
                    yy %= Ly
                elif xx >= Lx or yy >= Ly:
                    continue
                j = yy * Lx + xx
                if j != i:
                    bonds.add((min(i, j), max(i, j)))
    return sorted(bonds)


def class_pairs(Lx: int, Ly: int, periodic: bool):
    """For each displacement class, the ordered site pairs (i, j), i != j."""
    out = [[] for _ in CLASSES]
    Ns = Lx * Ly
    for i in range(Ns):
        for j in range(Ns):
            if i == j:
                continue
            ax = _min_image(j % Lx - i % Lx, Lx, periodic)
            ay = _min_image(j // Lx - i // Lx, Ly, periodic)
            for c, (cx, cy) in enumerate(CLASSES):
                if (ax, ay) == (cx, cy):
                    out[c].append((i, j))
    return out


class Sector:
    """Fixed-N sector of the truncated Bose-Hubbard lattice."""

    def __init__(self, Lx: int, Ly: int, d: int, N: int, periodic: bool, J: float, U: float):
        self.Lx, self.Ly, self.d, self.N, self.periodic, self.J, self.U = Lx, Ly, d, N, periodic, J, U
        self.Ns = Lx * Ly
        self.codes, self.occ = self._basis()
        self.dim = len(self.codes)
        self.pw = d ** np.arange(self.Ns, dtype=np.int64)
        self.bonds = lattice_bonds(Lx, Ly, periodic)
        self.H = self._hamiltonian()

    def _basis(self):
        """Every occupation tuple with sum N, by extending site by site the
        partial tuples whose remaining particles still fit."""
        d, Ns, N = self.d, self.Ns, self.N
        codes = np.zeros(1, dtype=np.int64)
        left = np.full(1, N, dtype=np.int64)
        for j in range(Ns):
            cap = (Ns - j - 1) * (d - 1)     # particles the later sites can still hold
            nc, nl = [], []
            for n in range(d):
                keep = (left >= n) & (left - n <= cap)
                nc.append(codes[keep] + n * d ** j)
                nl.append(left[keep] - n)
            codes, left = np.concatenate(nc), np.concatenate(nl)
        codes = np.sort(codes)
        occ = np.zeros((len(codes), Ns), dtype=np.int8)
        rem = codes.copy()
        for j in range(Ns):
            occ[:, j] = rem % d
            rem //= d
        assert (occ.sum(axis=1) == N).all()
        return codes, occ

    def index(self, codes: np.ndarray) -> np.ndarray:
        k = np.searchsorted(self.codes, codes)
        assert (self.codes[k] == codes).all()
        return k

    def _hamiltonian(self):
        """Diagonal U/2 sum n(n-1) plus -J for every hop a_i^+ a_j and
        a_j^+ a_i of every bond, assembled once from coordinate lists."""
        n = self.occ.astype(np.float64)
        rows = [np.arange(self.dim)]
        cols = [np.arange(self.dim)]
        vals = [0.5 * self.U * (n * (n - 1)).sum(axis=1)]
        for (i, j) in self.bonds:
            for (a, b) in ((i, j), (j, i)):
                src, dst, amp = self._hop_parts(a, b)
                rows.append(dst)
                cols.append(src)
                vals.append(-self.J * amp)
        H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.dim, self.dim))
        H.sum_duplicates()
        return H

    def fock(self, occ) -> np.ndarray:
        code = int(sum(int(n) * self.d ** j for j, n in enumerate(occ)))
        psi = np.zeros(self.dim, dtype=np.complex128)
        psi[self.index(np.array([code]))[0]] = 1.0
        return psi

    def _hop_parts(self, i: int, j: int):
        """(src, dst, amp) of a_i^+ a_j: basis states src with n_j >= 1 and
        n_i <= d-2 go to dst with amplitude sqrt(n_j) sqrt(n_i + 1)."""
        ni, nj = self.occ[:, i].astype(np.int64), self.occ[:, j].astype(np.int64)
        src = np.nonzero((nj >= 1) & (ni <= self.d - 2))[0]
        dst = self.index(self.codes[src] - self.pw[j] + self.pw[i])
        return src, dst, np.sqrt(nj[src]) * np.sqrt(ni[src] + 1.0)

    def observables(self, psi: np.ndarray, translation_invariant: bool = False) -> np.ndarray:
        """Slots 0..11 of the oracle's per-trajectory layout (exact values).
        translation_invariant: the state and H are invariant under lattice
        translations (periodic lattice, translation-invariant start), so the
        sum over ordered pairs divided by Ns equals the sum over the partners
        of site 0."""
        if not hasattr(self, "_pairs"):
            pairs = class_pairs(self.Lx, self.Ly, self.periodic)
            if translation_invariant:
                pairs = [[(i, j) for (i, j) in lst if i == 0] for lst in pairs]
            self._pairs = (translation_invariant, pairs, {})
        ti, pairs, cache = self._pairs
        assert ti == translation_invariant
        prob = np.abs(psi) ** 2
        n = self.occ.astype(np.float64)
        out = np.zeros(12)
        for c, lst in enumerate(pairs):
            for (i, j) in lst:
                if (i, j) not in cache:
                    cache[(i, j)] = self._hop_parts(i, j)
                src, dst, amp = cache[(i, j)]
                out[c] += np.real(np.sum(np.conj(psi[dst]) * psi[src] * amp))     # <a_i^+ a_j>
                out[5 + c] += prob @ (n[:, i] * n[:, j])
        norm = 1.0 if translation_invariant else self.Ns
        out[:10] /= norm
        out[10] = (prob @ n.sum(axis=1)) / self.Ns
        out[11] = np.vdot(psi, self.H @ psi).real / self.Ns
        return out

    def evolve(self, psi0: np.ndarray, times) -> np.ndarray:
        """psi(t) for each t of an evenly spaced grid starting at 0."""
        times = np.asarray(times, dtype=np.float64)
        A = (-1j) * self.H.astype(np.complex128)
        return expm_multiply(A, psi0, start=float(times[0]), stop=float(times[-1]), num=len(times), endpoint=True)


def mott_quench(Lx: int, Ly: int, d: int, periodic: bool, J: float, U: float, times):
    """Observables [len(times)][12] after the sudden quench of the
    unit-filling Mott state (one particle per site) to (J, U), and the
    sector dimension."""
    s = Sector(Lx, Ly, d, Lx * Ly, periodic, J, U)
    psi = s.evolve(s.fock([1] * s.Ns), times)
    return np.stack([s.observables(p, translation_invariant=periodic) for p in psi]), s.dim
