"""The packed Hermitian layout of the D = 256 path (2x2 clusters, d = 4):
the upper 16x16 tiles only, 34816 of 65536 entries per cluster.

Both layouts run the same stage kernels (the full layout writes every upper
tile and its conjugate transpose), so a packed plan must give, entry for
entry, the upper tiles of a full plan: sampling, commutator, mean fields,
RK4 over several calls and the observables (computed on an unpacked copy)
are compared bit for bit, and against the oracle at the parity tolerances."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")

TILES = [(I, J) for I in range(16) for J in range(I, 16)]


def unpack(pk):
    """[..., 34816] packed -> [..., 256, 256] Hermitian (numpy)."""
    lead = pk.shape[:-1]
    out = np.zeros(lead + (256, 256), dtype=pk.dtype)
    for k, (I, J) in enumerate(TILES):
        t = pk[..., k * 256:(k + 1) * 256].reshape(lead + (16, 16))
        out[..., 16 * I:16 * I + 16, 16 * J:16 * J + 16] = t
        if I != J:
            out[..., 16 * J:16 * J + 16, 16 * I:16 * I + 16] = np.conj(np.swapaxes(t, -1, -2))
    return out


def pack(full):
    lead = full.shape[:-2]
    out = np.zeros(lead + (len(TILES) * 256,), dtype=full.dtype)
    for k, (I, J) in enumerate(TILES):
        out[..., k * 256:(k + 1) * 256] = full[..., 16 * I:16 * I + 16, 16 * J:16 * J + 16].reshape(lead + (256,))
    return out


def _plans(L, n, dtype):
    kw = dict(d=4, periodic=True, J=1.0, U=5.0, dtype=dtype)
    full = cd.Plan(cd.Problem(L, L, 2, 2, **kw), n)
    pk = cd.Plan(cd.Problem(L, L, 2, 2, layout=cd.LAYOUT_PACKED, **kw), n)
    assert pk.state_shape() == (n, full.n_clusters, cd.PACKED_ELEMS)
    return full, pk


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_packed_sampling_commutator_fields(dtype):
    print("packed layout: sampling, commutator, fields, dtype", dtype, flush=True)
    n = 3
    full, pk = _plans(4, n, dtype)
    rf, rp = full.new_state(), pk.new_state()
    full.sample_noise(21, 4, rf)
    pk.sample_noise(21, 4, rp)
    assert torch.equal(torch.from_numpy(pack(rf.cpu().numpy())), rp.cpu())
    op = oracle.Problem(4, 4, 2, 2, d=4, periodic=True, J=1.0, U=5.0)
    _, r0 = oracle.sample(op, oracle.mott_tables(4), seed=21, traj_offset=4, n_traj=n)
    tol0 = 1e-14 if dtype == cd.F64 else 1e-6
    assert np.abs(unpack(rp.cpu().numpy()) - r0).max() <= tol0
    # evolve a little so that every entry is populated, then the commutator
    wf, wp = full.new_workspace(), pk.new_workspace()
    full.step_rk4(rf, wf, 0.02, 2)
    pk.step_rk4(rp, wp, 0.02, 2)
    Kf, Kp = torch.empty_like(rf), torch.empty_like(rp)
    full.commutator(rf, Kf, wf)
    pk.commutator(rp, Kp, wp)
    assert torch.equal(torch.from_numpy(pack(Kf.cpu().numpy())), Kp.cpu())
    Kref = oracle.rhs(op, unpack(rp.cpu().numpy()).astype(np.complex128))
    scale = np.abs(Kref).max()
    tolK = 1e-13 if dtype == cd.F64 else 1e-6
    assert np.abs(unpack(Kp.cpu().numpy()) - Kref).max() <= tolK * scale
    cdt = rf.dtype
    b_f, phi_f = (torch.empty(n, 16, dtype=cdt, device="cuda") for _ in range(2))
    b_p, phi_p = (torch.empty(n, 16, dtype=cdt, device="cuda") for _ in range(2))
    full.gather_boundary_fields(rf, b_f, phi_f)
    pk.gather_boundary_fields(rp, b_p, phi_p)
    assert torch.equal(b_f, b_p) and torch.equal(phi_f, phi_p)
    bref, phiref = oracle.fields(op, unpack(rp.cpu().numpy()).astype(np.complex128))
    assert np.abs(b_p.cpu().numpy() - bref).max() <= (1e-13 if dtype == cd.F64 else 1e-5)


@pytest.mark.parametrize("dtype", [cd.F64, cd.F32])
def test_packed_rk4_and_observables_match_full_and_oracle(dtype):
    """6x6 lattice (9 clusters), 5 trajectories, three calls of 3, 1 and 4
    steps with observables after each."""
    print("packed layout: RK4 and observables, dtype", dtype, flush=True)
    n = 5
    full, pk = _plans(6, n, dtype)
    rf, rp = full.new_state(), pk.new_state()
    wf, wp = full.new_workspace(), pk.new_workspace()
    full.sample_noise(8, 0, rf)
    pk.sample_noise(8, 0, rp)
    calls = (3, 1, 4)
    sf = torch.zeros(len(calls), cd.NOBS, 3, dtype=torch.float64, device="cuda")
    sp = torch.zeros_like(sf)
    pf = torch.zeros(len(calls), n, cd.NOBS, dtype=torch.float64, device="cuda")
    pp = torch.zeros_like(pf)
    for k, m in enumerate(calls):
        full.step_rk4(rf, wf, 0.01, m)
        pk.step_rk4(rp, wp, 0.01, m)
        full.accumulate_observables(rf, k, sf, wf, per_traj=pf[k])
        pk.accumulate_observables(rp, k, sp, wp, per_traj=pp[k])
    torch.cuda.synchronize()
    assert torch.equal(torch.from_numpy(pack(rf.cpu().numpy())), rp.cpu())
    assert torch.equal(pf, pp) and torch.equal(sf, sp)
    op = oracle.Problem(6, 6, 2, 2, d=4, periodic=True, J=1.0, U=5.0)
    steps = np.cumsum(calls).tolist()
    res = oracle.run(op, oracle.mott_tables(4), seed=8, traj_offset=0, n_traj=n, dt=0.01, n_steps=steps[-1],
                     record_steps=steps, want_rho=True)
    err = np.abs(pp.cpu().numpy().transpose(1, 0, 2)[:, :, :12] - res["obs"][:, :, :12]).max()
    serr = np.abs(unpack(rp.cpu().numpy()).astype(np.complex128) - res["rho"]).max()
    print(f"  observables {err:.2e}, state {serr:.2e}", flush=True)
    if dtype == cd.F64:
        assert err < 1e-11 and serr < 1e-12
    else:
        assert err < 2e-5 and serr < 2e-5
