"""Independent reference formulations used to pin the oracle.

Nothing here calls the oracle's arithmetic:
  * ``bh_hamiltonian`` builds the truncated Bose-Hubbard Hamiltonian of a small
    lattice directly in the occupation-number basis, matrix element by matrix
    element (no Kronecker products), and ``evolve`` propagates a density matrix
    with exp(-iHt) from an eigen-decomposition (exact diagonalisation).
  * ``DtwaR`` is the single-site SU(N) discrete truncated Wigner approximation
    written in the basis of the phase-space variables r^a themselves, with
    structure constants computed from the generator matrices; this is the
    Hamilton-equation form of the same dynamics (arXiv:2404.18594, App. B.2
    remarks that for unitary dynamics the variable form and the matrix form of
    the equations of motion are equivalent).
"""
from __future__ import annotations

import itertools

import numpy as np


def occupation_basis(n_sites: int, d: int):
    """All occupation tuples, first site most significant."""
    return list(itertools.product(range(d), repeat=n_sites))


def bh_hamiltonian(n_sites: int, bonds, d: int, J: float, U: float) -> np.ndarray:
    """H = -J sum_bonds (a_i^+ a_j + a_j^+ a_i) + U/2 sum_i n_i (n_i - 1), with
    occupations truncated to 0..d-1, in the occupation basis."""
    basis = occupation_basis(n_sites, d)
    index = {s: k for k, s in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)))
    for k, s in enumerate(basis):
        H[k, k] += 0.5 * U * sum(n * (n - 1) for n in s)
        for (i, j) in bonds:
            for (src, dst) in ((j, i), (i, j)):   # a_dst^+ a_src
                if s[src] == 0 or s[dst] == d - 1:
                    continue
                t = list(s)
                amp = np.sqrt(s[src]) * np.sqrt(s[dst] + 1)
                t[src] -= 1
                t[dst] += 1
                H[index[tuple(t)], k] += -J * amp
    return H


def single_site_op(n_sites: int, d: int, site: int, kind: str) -> np.ndarray:
    """a_site, a_site^+ or n_site in the occupation basis."""
    basis = occupation_basis(n_sites, d)
    index = {s: k for k, s in enumerate(basis)}
    O = np.zeros((len(basis), len(basis)))
    for k, s in enumerate(basis):
        n = s[site]
        if kind == "n":
            O[k, k] = n
        elif kind == "a" and n > 0:
            t = list(s); t[site] -= 1
            O[index[tuple(t)], k] = np.sqrt(n)
        elif kind == "adag" and n < d - 1:
            t = list(s); t[site] += 1
            O[index[tuple(t)], k] = np.sqrt(n + 1)
    return O


def product_fock(n_sites: int, d: int, occ) -> np.ndarray:
    basis = occupation_basis(n_sites, d)
    k = basis.index(tuple(occ))
    rho = np.zeros((len(basis), len(basis)), dtype=np.complex128)
    rho[k, k] = 1.0
    return rho


def evolve(H: np.ndarray, rho0: np.ndarray, t: float) -> np.ndarray:
    w, V = np.linalg.eigh(H)
    Ut = (V * np.exp(-1j * w * t)) @ V.conj().T
    return Ut @ rho0 @ Ut.conj().T


def structure_constants(T: np.ndarray) -> np.ndarray:
    """f_abc with [T_a, T_b] = 2i sum_c f_abc T_c for Tr(T_a T_b) = 2 delta_ab."""
    n = T.shape[0]
    f = np.zeros((n, n, n))
    for a in range(n):
        for b in range(n):
            C = T[a] @ T[b] - T[b] @ T[a]
            for c in range(n):
                f[a, b, c] = np.real(np.trace(C @ T[c]) / 4j)
    return f


class DtwaR:
    """Single-site SU(d) dTWA for the truncated Bose-Hubbard model on an
    Lx x Ly lattice, state = r[site][a].  A_j = I/d + (1/2) sum_a r^a T_a is
    never formed; the mean-field Hamiltonian of site j,
        H_j = U h - J (conj(phi_j) a + phi_j a^+),  phi_j = sum_k beta_k,
    is expanded as sum_b eta_b T_b (+ identity) and r evolves as
        dr^a/dt = 2 sum_{b,c} f_{bca} eta_b r^c,
    the image of dA/dt = -i[H_j, A_j] under A <-> r."""

    def __init__(self, Lx, Ly, periodic, d, J, U, T):
        self.Lx, self.Ly, self.periodic, self.d, self.J, self.U = Lx, Ly, periodic, d, J, U
        self.T = T
        self.f = structure_constants(T)
        a = np.zeros((d, d))
        for n in range(1, d):
            a[n - 1, n] = np.sqrt(n)
        self.a = a
        self.h = np.diag([0.5 * n * (n - 1) for n in range(d)])
        self.num = np.diag(np.arange(d, dtype=float))
        # beta = Tr(a A) = (1/2) sum_c r^c Tr(a T_c); n = Tr(n A)
        self.ca = 0.5 * np.array([np.trace(a @ Tc) for Tc in T])
        self.cn = 0.5 * np.array([np.real(np.trace(self.num @ Tc)) for Tc in T])
        self.n0 = np.trace(self.num) / d
        # eta for the U term and for unit fields: eta_b = (1/2) Tr(H T_b)
        self.eta_U = 0.5 * np.array([np.real(np.trace(U * self.h @ Tc)) for Tc in T])
        self.eta_a = 0.5 * np.array([np.trace(a @ Tc) for Tc in T])        # coefficient of conj(phi)
        self.eta_ad = 0.5 * np.array([np.trace(a.T @ Tc) for Tc in T])     # coefficient of phi
        Ns = Lx * Ly
        self.nbrs = []
        for j in range(Ns):
            x, y = j % Lx, j // Lx
            lst = []
            for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                xx, yy = x + dx, y + dy
                if periodic:
                    xx %= Lx; yy %= Ly
                elif not (0 <= xx < Lx and 0 <= yy < Ly):
                    continue
                lst.append(yy * Lx + xx)
            self.nbrs.append(lst)

    def beta(self, r):
        return r @ self.ca

    def rhs(self, r):
        beta = self.beta(r)
        phi = np.array([sum(beta[k] for k in nb) for nb in self.nbrs])
        eta = self.eta_U[None, :] - self.J * (np.conj(phi)[:, None] * self.eta_a[None, :] + phi[:, None] * self.eta_ad[None, :])
        eta = np.real(eta)
        return 2.0 * np.einsum("bca,jb,jc->ja", self.f, eta, r)

    def rk4(self, r, dt, n_steps):
        for _ in range(n_steps):
            k1 = self.rhs(r)
            k2 = self.rhs(r + 0.5 * dt * k1)
            k3 = self.rhs(r + 0.5 * dt * k2)
            k4 = self.rhs(r + dt * k3)
            r = r + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        return r

    def observables(self, r):
        """Pair sums over ordered pairs at minimum-image |dx|,|dy| classes
        (1,0),(0,1),(1,1),(2,0),(0,2) of Re conj(beta_i) beta_j and n_i n_j,
        divided by Ns, plus the mean density."""
        Lx, Ly = self.Lx, self.Ly
        Ns = Lx * Ly
        beta = self.beta(r)
        n = self.n0 + r @ self.cn
        classes = [(1, 0), (0, 1), (1, 1), (2, 0), (0, 2)]
        out = np.zeros(11)

        def mi(dd, L):
            if not self.periodic:
                return abs(dd)
            m = dd % L
            return min(m, L - m)

        for i in range(Ns):
            for j in range(Ns):
                if i == j:
                    continue
                c = (mi(j % Lx - i % Lx, Lx), mi(j // Lx - i // Lx, Ly))
                if c in classes:
                    k = classes.index(c)
                    out[k] += np.real(np.conj(beta[i]) * beta[j]) / Ns
                    out[5 + k] += n[i] * n[j] / Ns
        out[10] = n.mean()
        return out


# ---------------------------------------------------------------------------
# Spin-1/2 chains (App. A): basis state k has bit (n-1-i) of k set when site i
# is down, so site 0 is the most significant factor and |0> = |up>.
# ---------------------------------------------------------------------------

def ising_hamiltonian(n_sites: int, bonds, J: float, h: float) -> np.ndarray:
    """H = J sum_bonds s^z_i s^z_j + h sum_i s^x_i, element by element:
    s^z is diagonal (+1 up, -1 down), s^x flips one spin."""
    dim = 1 << n_sites
    H = np.zeros((dim, dim))
    for k in range(dim):
        z = [1 - 2 * ((k >> (n_sites - 1 - i)) & 1) for i in range(n_sites)]
        H[k, k] += J * sum(z[i] * z[j] for (i, j) in bonds)
        for i in range(n_sites):
            H[k ^ (1 << (n_sites - 1 - i)), k] += h
    return H


def spin_op(n_sites: int, site: int, kind: str) -> np.ndarray:
    """s^x, s^y or s^z of one site in the same basis."""
    dim = 1 << n_sites
    O = np.zeros((dim, dim), dtype=np.complex128)
    bit = 1 << (n_sites - 1 - site)
    for k in range(dim):
        down = (k & bit) != 0
        if kind == "z":
            O[k, k] = -1.0 if down else 1.0
        elif kind == "x":
            O[k ^ bit, k] = 1.0
        else:   # s^y |up> = i |down>, s^y |down> = -i |up>
            O[k ^ bit, k] = -1j if down else 1j
    return O


def spin_product_state(spins_up) -> np.ndarray:
    """|s_0 s_1 ...><...| with True for up."""
    n = len(spins_up)
    k = sum((0 if up else 1) << (n - 1 - i) for i, up in enumerate(spins_up))
    rho = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    rho[k, k] = 1.0
    return rho


def bloch_rhs(s: np.ndarray, nbrs, J: float, h: float) -> np.ndarray:
    """Classical spins s[j] = (s^x, s^y, s^z) of the single-site mean-field
    Ising chain: ds_j/dt = 2 B_j x s_j with B_j = (h, 0, J sum_k s^z_k) over the
    neighbours k of j (Heisenberg equation of a Pauli vector in the field B)."""
    B = np.zeros_like(s)
    B[:, 0] = h
    for j, nb in enumerate(nbrs):
        B[j, 2] = J * sum(s[k, 2] for k in nb)
    return 2.0 * np.cross(B, s)
