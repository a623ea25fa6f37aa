"""Plain FP64 CPU oracle of the cluster discrete truncated Wigner approximation
(C-dTWA, Nagao & Yunoki, arXiv:2404.18594) for the truncated Bose-Hubbard model.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously-correct
statement of what the GPU library computes.  Only ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark import it; the product path never
does, and the oracle imports nothing from the product package.

The arithmetic lives in ``cdtwa_oracle.c`` (dense Kronecker-built operators,
two plain matrix products per commutator, classical RK4); this module builds it
with gcc, loads it with ctypes and supplies the sampling tables computed from
the generator basis in ``su_n.py``.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
closed forms printed in the paper, exact diagonalisation, an independent
SU(3) dTWA in the r-basis and per-trajectory invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import su_n

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdtwa_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NOBS = 15
OBS_NAMES = [
    "csp_10", "csp_01", "csp_11", "csp_20", "csp_02",
    "nn_10", "nn_01", "nn_11", "nn_20", "nn_02",
    "density", "energy", "purity", "trace_dev", "herm_dev",
]
MAXD = 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int), ("Ly", ctypes.c_int), ("cx", ctypes.c_int), ("cy", ctypes.c_int),
                ("d", ctypes.c_int), ("periodic", ctypes.c_int), ("J", ctypes.c_double), ("U", ctypes.c_double),
                ("model", ctypes.c_int), ("h", ctypes.c_double), ("init_state", ctypes.c_int),
                ("gdeph", ctypes.c_double), ("gloss", ctypes.c_double)]


@dataclass(frozen=True)
class Problem:
    """Lattice Lx x Ly (site j = y*Lx + x), clusters cx x cy, local dimension d.
    model 0: H = -J sum_<ij>(a_i^+ a_j + h.c.) + U/2 sum_i n_i(n_i-1) (Sec. III Eq. (H_bose));
    model 1 (d = 2): H = J sum_<ij> s^z_i s^z_j + h sum_i s^x_i (App. A Eq. (Hising)).
    init_state 1 (model 1): Neel state, |up> where x+y is even.
    gdeph, gloss (model 0): rates of the local Lindblad channels L_j = n_j
    (dephasing) and L_j = a_j (loss) acting on every cluster matrix."""
    Lx: int
    Ly: int
    cx: int
    cy: int
    d: int = 3
    periodic: bool = True
    J: float = 1.0
    U: float = 5.0
    model: int = 0
    h: float = 0.0
    init_state: int = 0
    gdeph: float = 0.0
    gloss: float = 0.0

    def c(self) -> _Problem:
        return _Problem(self.Lx, self.Ly, self.cx, self.cy, self.d, int(self.periodic), self.J, self.U,
                        self.model, self.h, self.init_state, self.gdeph, self.gloss)

    @property
    def Ns(self) -> int:
        return self.Lx * self.Ly

    @property
    def nloc(self) -> int:
        return self.cx * self.cy

    @property
    def nc(self) -> int:
        return (self.Lx // self.cx) * (self.Ly // self.cy)

    @property
    def D(self) -> int:
        return self.d ** self.nloc


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER(_Problem)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        _lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
        _lib.orc_geometry.argtypes = [P, vp]
        _lib.orc_maps.argtypes = [P, vp, vp, vp, vp, vp]
        _lib.orc_operators.argtypes = [P, vp, vp, vp, vp]
        _lib.orc_sample.argtypes = [P, ctypes.c_int, vp, vp, vp, vp, ctypes.c_double, ctypes.c_uint64, i64, i64,
                                    vp, vp, ctypes.c_int]
        _lib.orc_build_rho.argtypes = [P, ctypes.c_int, vp, vp, vp, ctypes.c_double, vp, i64, vp]
        _lib.orc_fields.argtypes = [P, vp, i64, vp, vp]
        _lib.orc_rhs.argtypes = [P, vp, i64, vp, ctypes.c_int]
        _lib.orc_rk4.argtypes = [P, vp, i64, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        _lib.orc_observables.argtypes = [P, vp, i64, vp, ctypes.c_int]
        _lib.orc_run.argtypes = [P, ctypes.c_int, vp, vp, vp, vp, ctypes.c_double, ctypes.c_uint64, i64, i64,
                                 ctypes.c_double, ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, ctypes.c_int]
        _lib.orc_patch_samples.argtypes = [ctypes.c_int, vp, vp, vp, ctypes.c_uint64, i64, i64, vp]
        _lib.orc_rk4_schedule.argtypes = [P, vp, i64, ctypes.c_double, ctypes.c_int, vp, vp, ctypes.c_int]
        for f in ("orc_geometry", "orc_maps", "orc_operators", "orc_sample", "orc_build_rho", "orc_fields", "orc_rhs", "orc_rk4",
                  "orc_observables", "orc_run", "orc_patch_samples", "orc_rk4_schedule"):
            getattr(_lib, f).restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st: int, what: str):
    if st != 0:
        raise ValueError(f"oracle {what} failed with status {st}")


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox-4x32-10 block function (Salmon et al., SC'11)."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


@dataclass
class Tables:
    T: np.ndarray        # [n_gen][d][d] complex
    n_out: np.ndarray    # [n_gen]
    val: np.ndarray      # [n_gen][4]
    prob: np.ndarray     # [n_gen][4]
    thr: np.ndarray      # [n_gen][4] uint64
    g_norm: float

    @property
    def n_gen(self) -> int:
        return self.T.shape[0]


def mott_tables(d: int) -> Tables:
    """Sampling tables of the unit-filling Mott state |1> (Sec. III) in the
    basis of ``su_n.generators(d)``."""
    T = su_n.generators(d)
    n_out, val, prob, thr = su_n.sampling_tables(T, su_n.fock_state(d, 1))
    g_norm = float(np.real(np.trace(T[0] @ T[0])))
    return Tables(T, n_out, val, prob, thr, g_norm)


def neel_tables() -> list:
    """Sampling tables of the two Neel sublattices of App. A (spin 1/2,
    Pauli basis): class 0 |up> (s^z = +1), class 1 |down>; s^x and s^y are
    +-1 with probability 1/2, s^z is fixed."""
    T = su_n.generators(2)
    out = []
    for n in (0, 1):
        n_out, val, prob, thr = su_n.sampling_tables(T, su_n.fock_state(2, n))
        out.append(Tables(T, n_out, val, prob, thr, float(np.real(np.trace(T[0] @ T[0])))))
    return out


def _first(tb):
    return tb[0] if isinstance(tb, (list, tuple)) else tb


def _tab_args(tb):
    """Arrays for the C side: generators of the first table; outcome counts,
    values and thresholds of every site class stacked ([n_class][n_gen]...)."""
    tbs = list(tb) if isinstance(tb, (list, tuple)) else [tb]
    t0 = tbs[0]
    Tr = np.ascontiguousarray(np.stack([t0.T.real, t0.T.imag], axis=-1).astype(np.float64))
    n_out = np.ascontiguousarray(np.stack([t.n_out for t in tbs]).astype(np.int32))
    val = np.ascontiguousarray(np.stack([t.val for t in tbs]).astype(np.float64))
    thr = np.ascontiguousarray(np.stack([t.thr for t in tbs]).astype(np.uint64))
    return (Tr, n_out, val, thr)


def geometry(p: Problem):
    out = np.zeros(4, dtype=np.int32)
    _check(lib().orc_geometry(ctypes.byref(p.c()), _ptr(out)), "geometry")
    return dict(Ns=int(out[0]), nc=int(out[1]), nloc=int(out[2]), D=int(out[3]))


def maps(p: Problem):
    """site -> cluster, site -> local index, neighbour table [Ns][4] in the
    order (+x, -x, +y, -y), intra-cluster bonds as local pairs."""
    Ns = p.Ns
    sc = np.zeros(Ns, dtype=np.int32)
    sl = np.zeros(Ns, dtype=np.int32)
    nb = np.zeros((Ns, 4), dtype=np.int32)
    bonds = np.zeros((16, 2), dtype=np.int32)
    nbond = np.zeros(1, dtype=np.int32)
    _check(lib().orc_maps(ctypes.byref(p.c()), _ptr(sc), _ptr(sl), _ptr(nb), _ptr(bonds), _ptr(nbond)), "maps")
    return sc, sl, nb, bonds[: int(nbond[0])]


def operators(p: Problem):
    """Embedded a_l, a_l^dag, n_l ([nloc][D][D]) and Gamma^intra ([D][D])."""
    D, nl = p.D, p.nloc
    B = np.zeros((nl, D, D), dtype=np.complex128)
    Bd = np.zeros_like(B)
    N = np.zeros_like(B)
    H0 = np.zeros((D, D), dtype=np.complex128)
    _check(lib().orc_operators(ctypes.byref(p.c()), _ptr(B), _ptr(Bd), _ptr(N), _ptr(H0)), "operators")
    return B, Bd, N, H0


def sample(p: Problem, tb: Tables, seed: int, traj_offset: int, n_traj: int, nthreads: int = 0):
    """Noise codes [n_traj][Ns][n_gen] (index of the drawn eigenvalue) and the
    initial cluster matrices rho [n_traj][nc][D][D]."""
    codes = np.zeros((n_traj, p.Ns, _first(tb).n_gen), dtype=np.int8)
    rho = np.zeros((n_traj, p.nc, p.D, p.D), dtype=np.complex128)
    Tr, n_out, val, thr = _tab_args(tb)
    _check(lib().orc_sample(ctypes.byref(p.c()), _first(tb).n_gen, _ptr(Tr), _ptr(n_out), _ptr(val), _ptr(thr),
                            _first(tb).g_norm,
                            seed, traj_offset, n_traj, _ptr(codes), _ptr(rho), nthreads), "sample")
    return codes, rho


def build_rho(p: Problem, tb: Tables, codes: np.ndarray) -> np.ndarray:
    """Cluster matrices [n][nc][D][D] from given outcome indices [n][Ns][n_gen]."""
    codes = np.ascontiguousarray(codes, dtype=np.int8)
    n = codes.shape[0]
    rho = np.zeros((n, p.nc, p.D, p.D), dtype=np.complex128)
    Tr, n_out, val, _ = _tab_args(tb)
    _check(lib().orc_build_rho(ctypes.byref(p.c()), _first(tb).n_gen, _ptr(Tr), _ptr(n_out), _ptr(val),
                               _first(tb).g_norm,
                               _ptr(codes), n, _ptr(rho)), "build_rho")
    return rho


def fields(p: Problem, rho: np.ndarray):
    """Cluster mean fields b_j = Tr(a_j A_mu(j)) and boundary fields phi_j."""
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    n = rho.shape[0]
    b = np.zeros((n, p.Ns), dtype=np.complex128)
    phi = np.zeros_like(b)
    _check(lib().orc_fields(ctypes.byref(p.c()), _ptr(rho), n, _ptr(b), _ptr(phi)), "fields")
    return b, phi


def rhs(p: Problem, rho: np.ndarray, nthreads: int = 0) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    K = np.zeros_like(rho)
    _check(lib().orc_rhs(ctypes.byref(p.c()), _ptr(rho), rho.shape[0], _ptr(K), nthreads), "rhs")
    return K


def rk4(p: Problem, rho: np.ndarray, dt: float, n_steps: int, nthreads: int = 0) -> np.ndarray:
    out = np.array(rho, dtype=np.complex128, order="C", copy=True)
    _check(lib().orc_rk4(ctypes.byref(p.c()), _ptr(out), out.shape[0], dt, n_steps, nthreads), "rk4")
    return out


def rk4_schedule(p: Problem, rho: np.ndarray, dt: float, n_steps: int, c1_half, c2_half,
                 nthreads: int = 0) -> np.ndarray:
    """n_steps RK4 steps with time-dependent couplings: c1_half[k], c2_half[k]
    are (J, U) -- (J, h) for the Ising model -- at t0 + k dt/2, k = 0..2 n_steps."""
    c1 = np.ascontiguousarray(c1_half, dtype=np.float64)
    c2 = np.ascontiguousarray(c2_half, dtype=np.float64)
    if c1.shape != (2 * n_steps + 1,) or c2.shape != c1.shape:
        raise ValueError("schedules need 2*n_steps+1 half-step values")
    out = np.array(rho, dtype=np.complex128, order="C", copy=True)
    _check(lib().orc_rk4_schedule(ctypes.byref(p.c()), _ptr(out), out.shape[0], dt, n_steps, _ptr(c1), _ptr(c2),
                                  nthreads), "rk4_schedule")
    return out


def observables(p: Problem, rho: np.ndarray, nthreads: int = 0) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.complex128)
    obs = np.zeros((rho.shape[0], NOBS))
    _check(lib().orc_observables(ctypes.byref(p.c()), _ptr(rho), rho.shape[0], _ptr(obs), nthreads), "observables")
    return obs


def run(p: Problem, tb: Tables, seed: int, traj_offset: int, n_traj: int, dt: float, n_steps: int,
        record_steps, want_codes: bool = False, want_rho: bool = False, nthreads: int = 0):
    """Sample, integrate and record observables [n_traj][n_record][NOBS]."""
    rec = np.ascontiguousarray(np.asarray(record_steps, dtype=np.int32))
    obs = np.zeros((n_traj, len(rec), NOBS))
    codes = np.zeros((n_traj, p.Ns, _first(tb).n_gen), dtype=np.int8) if want_codes else None
    rho = np.zeros((n_traj, p.nc, p.D, p.D), dtype=np.complex128) if want_rho else None
    Tr, n_out, val, thr = _tab_args(tb)
    _check(lib().orc_run(ctypes.byref(p.c()), _first(tb).n_gen, _ptr(Tr), _ptr(n_out), _ptr(val), _ptr(thr),
                         _first(tb).g_norm,
                         seed, traj_offset, n_traj, dt, n_steps, _ptr(rec), len(rec), _ptr(obs), _ptr(codes),
                         _ptr(rho), nthreads), "run")
    out = {"obs": obs}
    if want_codes:
        out["codes"] = codes
    if want_rho:
        out["rho"] = rho
    return out
