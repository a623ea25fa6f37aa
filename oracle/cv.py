"""Oracle of the learned control variate (an addition to the paper's method:
the paper estimates observables by plain trajectory averages, Sec. II).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  Plain numpy in FP64:

* patch features and per-cluster targets of the nearest-neighbour
  correlation (Sec. III definition of C^sp at distance one);
* i.i.d. patch features from Philox-4x32-10 (Salmon et al., SC'11) with the
  counter layout of the library's patch sampler;
* the network 128 -> 256 -> 256 -> 64 (ReLU), its mean-squared-error loss and
  hand-written backpropagation, with an optional rounding of every matrix
  product operand to BF16 (nearest, ties to even) so that it sees the same
  operands as the device products (which accumulate in FP32; here FP64);
* Adam (Kingma & Ba, ICLR 2015) with bias correction.

Pins (tests/test_oracle_cv.py): BF16 rounding against torch's own
conversion; backpropagation against central finite differences; Adam against
its closed forms (first step, constant gradient); features against a
roll-based patch extraction; targets summed over clusters against the
oracle's C^sp observables; sampler frequencies against the tomography
probabilities.  The trained network itself is parity unpinned (training is
not deterministic across precisions); only the estimator's unbiasedness is
checked, statistically.
"""
from __future__ import annotations

import numpy as np

from . import Problem, Tables, _check, _ptr, _tab_args, fields, lib, maps, operators, philox4x32_10

NI, NH, NO = 128, 256, 64
SHAPES = [("W1", (NI, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NO)), ("b3", (NO,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params: np.ndarray) -> dict:
    """Split the flat parameter vector (W1, b1, W2, b2, W3, b3; W[in][out])."""
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(params[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_bits(x) -> np.ndarray:
    """BF16 bit patterns of x rounded first to FP32, then to BF16 (nearest,
    ties to even; the upper 16 bits of the FP32 pattern after adding half an
    ulp of BF16 plus the tie-breaking bit)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16(x) -> np.ndarray:
    """Values of x rounded to BF16, as FP64."""
    bits = bf16_bits(x).astype(np.uint32) << 16
    return bits.view(np.float32).astype(np.float64)


def _q(rounding: bool):
    return bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))


def forward(params: np.ndarray, x: np.ndarray, rounding: bool = True):
    """y = relu(relu(x W1 + b1) W2 + b2) W3 + b3 with the product operands
    rounded to BF16 when `rounding`; returns y and the cache for backward."""
    P = unpack(params)
    q = _q(rounding)
    x0 = q(x)
    z1 = x0 @ q(P["W1"]) + P["b1"]
    a1 = q(np.maximum(z1, 0.0))
    z2 = a1 @ q(P["W2"]) + P["b2"]
    a2 = q(np.maximum(z2, 0.0))
    y = a2 @ q(P["W3"]) + P["b3"]
    return y, dict(P=P, x0=x0, z1=z1, a1=a1, z2=z2, a2=a2, rounding=rounding)


def loss(y: np.ndarray, target: np.ndarray) -> float:
    """Mean over all entries of (y - target)^2."""
    return float(np.mean((y - target) ** 2))


def backward(cache: dict, y: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Gradient of `loss` with respect to the parameters, by the chain rule
    through the three layers; the operands of the products are rounded like
    in the forward pass when the cache says so."""
    P, q = cache["P"], _q(cache["rounding"])
    n = y.shape[0]
    dy = 2.0 * (y - target) / (n * NO)
    dyq = q(dy)
    g = {}
    g["W3"] = cache["a2"].T @ dyq
    g["b3"] = dy.sum(axis=0)
    da2 = dyq @ q(P["W3"]).T
    dz2 = da2 * (cache["z2"] > 0)
    dz2q = q(dz2)
    g["W2"] = cache["a1"].T @ dz2q
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2q @ q(P["W2"]).T
    dz1 = da1 * (cache["z1"] > 0)
    dz1q = q(dz1)
    g["W1"] = cache["x0"].T @ dz1q
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def adam(params, grad, m, v, lr: float, step: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step; returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Patches, features and targets
# ---------------------------------------------------------------------------
def patch_sites(p: Problem, mu: int):
    """The 16 sites (y-major: s = 4 (y - y0 + 1) + (x - x0 + 1)) of the 4x4
    patch around 2x2 cluster mu, -1 for a site outside an open lattice."""
    ncx = p.Lx // p.cx
    x0, y0 = (mu % ncx) * p.cx, (mu // ncx) * p.cy
    out = []
    for s in range(16):
        x, y = x0 - 1 + s % 4, y0 - 1 + s // 4
        if p.periodic:
            out.append((y % p.Ly) * p.Lx + (x % p.Lx))
        else:
            out.append(y * p.Lx + x if 0 <= x < p.Lx and 0 <= y < p.Ly else -1)
    return out


def features(p: Problem, tb: Tables, codes: np.ndarray) -> np.ndarray:
    """[n_traj * nc][16 * n_gen] (FP32) patch features: r^a of every patch site."""
    n = codes.shape[0]
    ng = tb.n_gen
    out = np.zeros((n, p.nc, 16 * ng))
    for mu in range(p.nc):
        for s, j in enumerate(patch_sites(p, mu)):
            if j < 0:
                continue
            for a in range(ng):
                out[:, mu, s * ng + a] = tb.val[a][codes[:, j, a]]
    return out.reshape(n * p.nc, 16 * ng).astype(np.float32)


def targets(p: Problem, rho: np.ndarray) -> np.ndarray:
    """[n_traj][nc] t_mu = sum over sites i of cluster mu of
    Re<a_i^+ a_(i+x)> + Re<a_i^+ a_(i+y)>: Tr(a_i^+ a_j rho_mu) when j is in
    mu, Re(conj(b_i) b_j) with b_k = Tr(a_k rho_nu(k)) otherwise."""
    sc, sl, _, _ = maps(p)
    B, Bd, _, _ = operators(p)
    b, _ = fields(p, rho)
    n = rho.shape[0]
    out = np.zeros((n, p.nc))
    for i in range(p.Ns):
        xi, yi = i % p.Lx, i // p.Lx
        mu = sc[i]
        for dx, dy in ((1, 0), (0, 1)):
            xj, yj = xi + dx, yi + dy
            if p.periodic:
                xj, yj = xj % p.Lx, yj % p.Ly
            elif xj >= p.Lx or yj >= p.Ly:
                continue
            j = yj * p.Lx + xj
            if sc[j] == mu:
                op = Bd[sl[i]] @ B[sl[j]]
                val = np.einsum("pq,tqp->t", op, rho[:, mu])
            else:
                val = np.conj(b[:, i]) * b[:, j]
            out[:, mu] += val.real
    return out


def sample_patch_features(tb: Tables, seed: int, first: int, n: int) -> np.ndarray:
    """Features [n][16 * n_gen] (FP32) of i.i.d. patches first..first+n-1:
    patch p, site s, generator a from Philox-4x32-10 with counter
    (a/4, s, p_lo, p_hi), key (seed_lo, seed_hi ^ 0x5bd1e995), word a % 4;
    outcome = first eigenvalue index o with x < thr[a][o] (last one if none).
    The loop runs in the oracle's C code (orc_patch_samples)."""
    out = np.zeros((n, 16, tb.n_gen))
    _, n_out, val, thr = _tab_args(tb)
    _check(lib().orc_patch_samples(tb.n_gen, _ptr(n_out), _ptr(val), _ptr(thr), seed, first, n, _ptr(out)),
           "patch_samples")
    return out.reshape(n, 16 * tb.n_gen).astype(np.float32)


def sample_patch_features_py(tb: Tables, seed: int, first: int, n: int) -> np.ndarray:
    """The same draws written out in Python one Philox block at a time (a
    second statement of the counter layout, for small n)."""
    ng = tb.n_gen
    out = np.zeros((n, 16 * ng))
    k = [seed & 0xFFFFFFFF, ((seed >> 32) & 0xFFFFFFFF) ^ 0x5BD1E995]
    for r in range(n):
        pi = first + r
        for s in range(16):
            for blk in range((ng + 3) // 4):
                w = philox4x32_10([blk, s, pi & 0xFFFFFFFF, (pi >> 32) & 0xFFFFFFFF], k)
                for a in range(4 * blk, min(ng, 4 * blk + 4)):
                    x = int(w[a % 4])
                    o = 0
                    while o < tb.n_out[a] - 1 and not (x < int(tb.thr[a][o])):
                        o += 1
                    out[r, s * ng + a] = tb.val[a][o]
    return out.astype(np.float32)
