"""Pins of the oracle's onsite algebra and discrete sampling against what the
paper prints (App. B.1) and against closed forms (arXiv:2404.18594)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import su_n
from conftest import read_golden


def test_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


@pytest.mark.parametrize("d", [2, 3, 4])
def test_generators_hermitian_traceless_orthonormal(d):
    T = su_n.generators(d)
    assert T.shape == (d * d - 1, d, d)
    for a in range(T.shape[0]):
        assert np.allclose(T[a], T[a].conj().T)
        assert abs(np.trace(T[a])) < 1e-14
    G = np.einsum("aij,bji->ab", T, T)
    assert np.allclose(G, 2 * np.eye(T.shape[0]), atol=1e-14)
    # they span the traceless Hermitian matrices
    M = np.array([np.concatenate([t.real.ravel(), t.imag.ravel()]) for t in T])
    assert np.linalg.matrix_rank(M) == d * d - 1


def test_cartan_weights_label_fock_states():
    T = su_n.generators(3)
    for fock, w3, w8 in read_golden("su3_cartan_weights.txt"):
        n = int(fock)
        assert np.isclose(T[2][n, n].real, float(w3))
        assert np.isclose(T[7][n, n].real, float(w8) / np.sqrt(3))
    # T_3 and T_8 are diagonal
    for a in (2, 7):
        assert np.allclose(T[a], np.diag(np.diag(T[a])))


def _parse_matrices(rows):
    mats, cur, name = {}, [], None
    for r in rows:
        if len(r) == 1 and not r[0][0].isdigit() and r[0] != "sqrt2":
            if name:
                mats[name] = np.array(cur)
            name, cur = r[0], []
        else:
            cur.append([np.sqrt(2) if x == "sqrt2" else float(x) for x in r])
    mats[name] = np.array(cur)
    return mats


def test_boson_matrices_match_paper():
    mats = _parse_matrices(read_golden("boson_matrices_d3.txt"))
    a, ad, num, h = su_n.boson_ops(3)
    assert np.allclose(a, mats["a"])
    assert np.allclose(ad, mats["adag"])
    assert np.allclose(h, mats["Hint"])          # U h = H_int
    # the oracle's embedded operators agree for a single site
    B, Bd, N, H0 = oracle.operators(oracle.Problem(1, 1, 1, 1, d=3, periodic=False, J=1.0, U=1.0))
    assert np.allclose(B[0], mats["a"]) and np.allclose(Bd[0], mats["adag"])
    assert np.allclose(N[0], np.diag([0, 1, 2])) and np.allclose(H0, mats["Hint"])


def test_mott_fluctuating_generators():
    g = {r[0]: r[1:] for r in read_golden("mott_sampling.txt")}
    fluct = sorted(int(x) for x in g["fluctuating"])
    tb = oracle.mott_tables(3)
    got = [a + 1 for a in range(8) if np.count_nonzero(tb.prob[a, : tb.n_out[a]] > 1e-12) > 1]
    assert got == fluct
    assert len(got) == int(g["noises_per_site"][0])
    assert 4 * len(got) == int(g["noises_per_2x2_cluster"][0])
    # fluctuating values are +-1 with probability 1/2; fixed values 0 (T3,T4,T5) and 2/sqrt(3) (T8)
    for a in range(8):
        vals = tb.val[a, : tb.n_out[a]]
        probs = tb.prob[a, : tb.n_out[a]]
        if a + 1 in fluct:
            assert np.allclose(vals[probs > 1e-12], [-1, 1])
            assert np.allclose(probs[probs > 1e-12], [0.5, 0.5])
        else:
            (only,) = vals[probs > 1e-12]
            assert np.isclose(only, 2 / np.sqrt(3) if a == 7 else 0.0)


def _enumerate_site(tb):
    """All outcome combinations with their probabilities for one site."""
    choices = []
    for a in range(tb.n_gen):
        choices.append([(n, tb.prob[a, n]) for n in range(tb.n_out[a]) if tb.prob[a, n] > 1e-12])
    for combo in itertools.product(*choices):
        w = np.prod([c[1] for c in combo])
        yield np.array([c[0] for c in combo], dtype=np.int8), w


@pytest.mark.parametrize("d", [2, 3, 4])
def test_mott_reconstruction_and_per_sample_invariants(d):
    """E[A_j] = |1><1| over the exact noise distribution (App. B.1), and every
    sample has Tr A = 1, Tr A^2 = (1 + (N-1) ... ) fixed, diag = e_1."""
    tb = oracle.mott_tables(d)
    p = oracle.Problem(1, 1, 1, 1, d=d, periodic=False)
    mean = np.zeros((d, d), dtype=complex)
    total = 0.0
    purities, spectra = set(), []
    for codes, w in _enumerate_site(tb):
        A = oracle.build_rho(p, tb, codes[None, None, :])[0, 0]
        mean += w * A
        total += w
        assert np.isclose(np.trace(A), 1.0)
        assert np.allclose(np.diag(A).real, np.eye(d)[1])
        purities.add(round(float(np.real(np.trace(A @ A))), 10))
        spectra.append(np.sort(np.linalg.eigvalsh(A)))
    assert np.isclose(total, 1.0)
    assert np.allclose(mean, np.diag(np.eye(d)[1]), atol=1e-14)
    assert len(purities) == 1
    if d == 3:
        # with the paper's basis every sample has spectrum {(1-sqrt5)/2, 0, (1+sqrt5)/2}, Tr A^2 = 3
        assert purities == {3.0}
        for s in spectra:
            assert np.allclose(s, [(1 - np.sqrt(5)) / 2, 0, (1 + np.sqrt(5)) / 2])


def test_symmetric_ordered_moment():
    """E |<a>|^2 = <(a^+ a + a a^+)/2> = 3/2 in |1> (Weyl-ordered second moment)."""
    tb = oracle.mott_tables(3)
    p = oracle.Problem(1, 1, 1, 1, d=3, periodic=False)
    a = su_n.boson_ops(3)[0]
    m2 = 0.0
    for codes, w in _enumerate_site(tb):
        A = oracle.build_rho(p, tb, codes[None, None, :])[0, 0]
        m2 += w * abs(np.trace(a @ A)) ** 2
    assert np.isclose(m2, 1.5)


def test_sampling_statistics_and_determinism():
    p = oracle.Problem(4, 4, 2, 2)
    tb = oracle.mott_tables(3)
    codes, rho = oracle.sample(p, tb, seed=7, traj_offset=0, n_traj=400)
    # fixed generators constant, fluctuating ones fair
    for a in range(8):
        c = codes[:, :, a].ravel()
        if a + 1 in (1, 2, 6, 7):
            assert set(np.unique(c)) == {0, 2}
            frac = np.mean(c == 2)
            n = c.size
            assert abs(frac - 0.5) < 4 * np.sqrt(0.25 / n)
        else:
            assert len(np.unique(c)) == 1
    # generators of one site are not correlated with each other
    s1 = 2.0 * (codes[:, :, 0] == 2) - 1
    s2 = 2.0 * (codes[:, :, 1] == 2) - 1
    assert abs(np.mean(s1 * s2)) < 4 / np.sqrt(s1.size)
    # counter-based: a trajectory depends only on (seed, global index)
    codes2, rho2 = oracle.sample(p, tb, seed=7, traj_offset=100, n_traj=3)
    assert np.array_equal(codes2, codes[100:103])
    assert np.array_equal(rho2, rho[100:103])
    codes3, _ = oracle.sample(p, tb, seed=8, traj_offset=100, n_traj=3)
    assert not np.array_equal(codes3, codes2)


def test_cluster_product_reconstructs_initial_state():
    """Enumerating all 2^16 noise configurations of a 2x2 cluster gives
    E[A_1 (x) A_2 (x) A_3 (x) A_4] = |1111><1111| (App. B.1, A_tot), and every
    configuration has Tr rho_C^2 = 3^4."""
    p = oracle.Problem(2, 2, 2, 2, periodic=False)
    tb = oracle.mott_tables(3)
    site_cfgs = list(_enumerate_site(tb))
    assert len(site_cfgs) == 16
    mean = np.zeros((81, 81), dtype=complex)
    batch, weights = [], []
    for combo in itertools.product(range(16), repeat=4):
        batch.append(np.stack([site_cfgs[k][0] for k in combo]))
        weights.append(np.prod([site_cfgs[k][1] for k in combo]))
        if len(batch) == 4096:
            rho = oracle.build_rho(p, tb, np.array(batch))[:, 0]
            mean += np.einsum("n,nij->ij", np.array(weights), rho)
            pur = np.einsum("nij,nji->n", rho, rho).real
            assert np.allclose(pur, 81.0)
            batch, weights = [], []
    target = np.zeros((81, 81)); target[40, 40] = 1.0   # |1111> = index 1*27+1*9+1*3+1
    assert np.allclose(mean, target, atol=1e-12)
