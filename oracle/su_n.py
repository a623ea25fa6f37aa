"""Onsite algebra of the oracle: SU(d) generator bases, truncated boson
operators and the discrete (tomographic) sampling tables.

TEST INFRASTRUCTURE ONLY -- part of the CPU oracle, see ``oracle/__init__.py``.

Sources (arXiv:2404.18594):
  * App. B.1: the eight 3x3 matrices T_1..T_8 used for n_max = 2 and the
    onsite ansatz A_j = I/3 + (1/2) sum_a r^a_j T_a; the Cartan weights of
    (T_3, T_8) label Fock states |0>, |1>, |2>.
  * App. B.1: the truncated boson matrices a, a^dagger and H_int = diag(0,0,U).
  * Sec. II: A_j = N^-1 I + g^-1 sum_a r^a s^a with g = Tr (s^a)^2, and the
    tomography rule: r^a takes eigenvalue lambda_n of s^a with probability
    tr[rho_j |phi_n><phi_n|] (App. B.1 gives the same rule for SU(3)).

Readings where the paper gives no basis: d = 2 uses the Pauli matrices (the
basis of the Ising appendix, App. A); d = 4 uses the generalised Gell-Mann
matrices normalised to Tr(T_a T_b) = 2 delta_ab, the normalisation of the
paper's SU(3) set.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)
SQ3 = np.sqrt(3.0)


def paper_su3_generators() -> np.ndarray:
    """T_1..T_8 exactly as printed in App. B.1 (index 0 holds T_1)."""
    T = np.zeros((8, 3, 3), dtype=np.complex128)
    T[0] = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]]) / SQ2
    T[1] = np.array([[0, -1j, 0], [1j, 0, -1j], [0, 1j, 0]]) / SQ2
    T[2] = np.array([[1, 0, 0], [0, 0, 0], [0, 0, -1]])
    T[3] = np.array([[0, 0, 1], [0, 0, 0], [1, 0, 0]])
    T[4] = np.array([[0, 0, -1j], [0, 0, 0], [1j, 0, 0]])
    T[5] = np.array([[0, -1, 0], [-1, 0, 1], [0, 1, 0]]) / SQ2
    T[6] = np.array([[0, 1j, 0], [-1j, 0, -1j], [0, 1j, 0]]) / SQ2
    T[7] = np.array([[-1, 0, 0], [0, 2, 0], [0, 0, -1]]) / SQ3
    return T


def pauli_generators() -> np.ndarray:
    """sigma_x, sigma_y, sigma_z (App. A works in this basis)."""
    return np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)


def gell_mann_generators(d: int) -> np.ndarray:
    """Generalised Gell-Mann basis of su(d), Tr(T_a T_b) = 2 delta_ab.

    Order: for each pair j<k (lexicographic) the symmetric X_jk then the
    antisymmetric Y_jk, followed by the d-1 diagonal matrices."""
    mats = []
    for j in range(d):
        for k in range(j + 1, d):
            X = np.zeros((d, d), dtype=np.complex128)
            X[j, k] = X[k, j] = 1.0
            Y = np.zeros((d, d), dtype=np.complex128)
            Y[j, k] = -1j
            Y[k, j] = 1j
            mats += [X, Y]
    for m in range(1, d):
        Z = np.zeros((d, d), dtype=np.complex128)
        for i in range(m):
            Z[i, i] = 1.0
        Z[m, m] = -m
        Z *= np.sqrt(2.0 / (m * (m + 1)))
        mats.append(Z)
    return np.array(mats)


def generators(d: int) -> np.ndarray:
    if d == 2:
        return pauli_generators()
    if d == 3:
        return paper_su3_generators()
    if d == 4:
        return gell_mann_generators(4)
    raise ValueError(f"unsupported local dimension d={d}")


def boson_ops(d: int):
    """a = sum_n sqrt(n)|n-1><n|, a^dagger, n, and h = n(n-1)/2 so that U*h is
    the interaction term U/2 a^dag a^dag a a of Sec. III Eq. (H_bose)."""
    a = np.zeros((d, d))
    for n in range(1, d):
        a[n - 1, n] = np.sqrt(n)
    num = np.diag(np.arange(d, dtype=float))
    h = np.diag([0.5 * n * (n - 1) for n in range(d)])
    return a, a.T.copy(), num, h


def fock_state(d: int, n: int) -> np.ndarray:
    rho = np.zeros((d, d), dtype=np.complex128)
    rho[n, n] = 1.0
    return rho


def sampling_tables(T: np.ndarray, rho: np.ndarray, tol: float = 1e-9):
    """Tomographic sampling rule for one site in state rho.

    For each generator T_a: the distinct eigenvalues (ascending) and the
    probability of each, p(lambda) = tr[rho P_lambda] with P_lambda the
    eigenprojector (the sum over eigenvectors of one eigenvalue; for a
    non-degenerate eigenvalue this is the paper's tr[rho |phi_n><phi_n|]).
    Returns (n_out[a], val[a, n], prob[a, n], thr[a, n]) with
    thr = round(2^32 * cumulative probability), last entry 2^32."""
    n_gen, d, _ = T.shape
    n_out = np.zeros(n_gen, dtype=np.int32)
    val = np.zeros((n_gen, 4))
    prob = np.zeros((n_gen, 4))
    thr = np.full((n_gen, 4), 1 << 32, dtype=np.uint64)
    for a in range(n_gen):
        w, V = np.linalg.eigh(T[a])
        groups: list[list[int]] = []
        for i in range(d):
            if groups and abs(w[i] - w[groups[-1][0]]) < tol:
                groups[-1].append(i)
            else:
                groups.append([i])
        n_out[a] = len(groups)
        cum = 0.0
        for n, grp in enumerate(groups):
            P = sum(np.outer(V[:, i], V[:, i].conj()) for i in grp)
            p = float(np.real(np.trace(rho @ P)))
            val[a, n] = float(np.mean(w[grp]))
            prob[a, n] = p
            cum += p
            thr[a, n] = np.uint64(min(1 << 32, int(round(cum * 2.0 ** 32))))
        thr[a, n_out[a] - 1] = np.uint64(1 << 32)
    return n_out, val, prob, thr
