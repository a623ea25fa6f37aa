"""The compensated FP32 state of the D = 256 path (2x2 clusters, d = 4):
cdtwa_step_rk4_compensated carries FP32 rho and its FP32 low parts
(packed), and forms rho + lo + increment with TwoSum at the end of each RK4
step.

Checked: a first step from zero low parts rounds rho exactly as the plain
FP32 step (bit for bit) and leaves the exact rounding error, within half
an ulp, in the low parts; several calls match the FP64 oracle with
rho + lo, the packed layout agreeing with the full one bit for bit; and
the entry point rejects plans it does not serve."""
import ctypes

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


def _plan(L, n, layout, dtype=None):
    prob = cd.Problem(L, L, 2, 2, d=4, periodic=True, J=1.0, U=5.0, dtype=cd.F32 if dtype is None else dtype,
                      layout=layout)
    return cd.Plan(prob, n)


def _packed_np(plan, rho):
    r = rho.cpu().numpy()
    return r if plan.problem.layout == cd.LAYOUT_PACKED else pack(r)


@pytest.mark.parametrize("layout", [cd.LAYOUT_FULL, cd.LAYOUT_PACKED])
def test_first_step_rounds_like_the_plain_step(layout):
    """From zero low parts the stages see the same FP32 rho, so the rounded
    sum equals the plain step's rho and the low part is its exact error."""
    print("compensated: first step, layout", layout, flush=True)
    n = 3
    plan = _plan(4, n, layout)
    r_plain, r_comp = plan.new_state(), plan.new_state()
    plan.sample_noise(5, 2, r_plain)
    r_comp.copy_(r_plain)
    r0 = _packed_np(plan, r_plain)
    lo = plan.new_low_parts()
    ws = plan.new_workspace()
    plan.step_rk4(r_plain, ws, 0.01, 1)
    plan.step_rk4_compensated(r_comp, lo, ws, 0.01, 1)
    torch.cuda.synchronize()
    assert torch.equal(r_plain, r_comp)
    hi = _packed_np(plan, r_comp)
    lo_np = lo.cpu().numpy()
    for part in (np.real, np.imag):
        h, low = part(hi).astype(np.float32), part(lo_np).astype(np.float32)
        # round to nearest: the error is at most half the spacing at hi
        assert (np.abs(low) <= 0.5 * np.spacing(np.abs(h))).all()
    live = np.count_nonzero(lo_np) / max(np.count_nonzero(hi), 1)
    print(f"  nonzero low parts: {live:.2f} of the nonzero entries", flush=True)
    assert live > 0.1                                      # the compensation is live
    assert not np.array_equal(hi, r0)


def test_compensated_rk4_matches_oracle_and_layouts_agree():
    """6x6 lattice (9 clusters), 5 trajectories, calls of 3, 1 and 4 steps;
    rho + lo against the oracle's FP64 RK4, observables of rho against the
    oracle's, and the packed plan against the full one bit for bit."""
    print("compensated: RK4 against the oracle, both layouts", flush=True)
    n = 5
    full, pk = _plan(6, n, cd.LAYOUT_FULL), _plan(6, n, cd.LAYOUT_PACKED)
    rf, rp = full.new_state(), pk.new_state()
    lf, lp = full.new_low_parts(), pk.new_low_parts()
    wf, wp = full.new_workspace(), pk.new_workspace()
    full.sample_noise(8, 0, rf)
    pk.sample_noise(8, 0, rp)
    calls = (3, 1, 4)
    pp = torch.zeros(len(calls), n, cd.NOBS, dtype=torch.float64, device="cuda")
    sp = torch.zeros(len(calls), cd.NOBS, 3, dtype=torch.float64, device="cuda")
    for k, m in enumerate(calls):
        full.step_rk4_compensated(rf, lf, wf, 0.01, m)
        pk.step_rk4_compensated(rp, lp, wp, 0.01, m)
        pk.accumulate_observables(rp, k, sp, wp, per_traj=pp[k])
    torch.cuda.synchronize()
    assert torch.equal(torch.from_numpy(pack(rf.cpu().numpy())), rp.cpu())
    assert torch.equal(lf, lp)
    op = oracle.Problem(6, 6, 2, 2, d=4, periodic=True, J=1.0, U=5.0)
    steps = np.cumsum(calls).tolist()
    res = oracle.run(op, oracle.mott_tables(4), seed=8, traj_offset=0, n_traj=n, dt=0.01, n_steps=steps[-1],
                     record_steps=steps, want_rho=True)
    state = unpack(rp.cpu().numpy().astype(np.complex128) + lp.cpu().numpy().astype(np.complex128))
    serr = np.abs(state - res["rho"]).max()
    herr = np.abs(unpack(rp.cpu().numpy()).astype(np.complex128) - res["rho"]).max()
    oerr = np.abs(pp.cpu().numpy().transpose(1, 0, 2)[:, :, :12] - res["obs"][:, :, :12]).max()
    print(f"  state rho + lo {serr:.2e} (rho alone {herr:.2e}), observables {oerr:.2e}", flush=True)
    assert serr < 2e-5 and herr < 2e-5 and oerr < 2e-5


def test_zero_steps_and_rejections():
    print("compensated: zero steps and rejected calls", flush=True)
    plan = _plan(4, 2, cd.LAYOUT_PACKED)
    rho, lo, ws = plan.new_state(), plan.new_low_parts(), plan.new_workspace()
    plan.sample_noise(1, 0, rho)
    before = rho.clone()
    plan.step_rk4_compensated(rho, lo, ws, 0.01, 0)
    torch.cuda.synchronize()
    assert torch.equal(rho, before) and not lo.any()
    with pytest.raises(cd.CdtwaError):                      # low parts of the wrong shape
        plan.step_rk4_compensated(rho, lo[:1], ws, 0.01, 1)
    lib = cd.library()
    h = plan._h
    assert lib.cdtwa_step_rk4_compensated(h, ctypes.c_void_p(rho.data_ptr()), None,
                                          ctypes.c_void_p(ws.data_ptr()), 0.01, 1, None) == -1
    assert lib.cdtwa_step_rk4_compensated(h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(lo.data_ptr()),
                                          ctypes.c_void_p(ws.data_ptr()), float("nan"), 1, None) == -1
    torch.cuda.synchronize()
    assert torch.equal(rho, before) and not lo.any()
    # FP64 state, and D = 81: not served (CDTWA_EUNSUPPORTED before any launch)
    for other in (_plan(4, 2, cd.LAYOUT_PACKED, cd.F64),
                  cd.Plan(cd.Problem(4, 4, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F32), 2)):
        r, w = other.new_state(), other.new_workspace()
        fake_lo = torch.zeros(2, other.n_clusters, cd.PACKED_ELEMS, dtype=torch.complex64, device="cuda")
        st = lib.cdtwa_step_rk4_compensated(other._h, ctypes.c_void_p(r.data_ptr()),
                                            ctypes.c_void_p(fake_lo.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                            0.01, 1, None)
        assert st == -2
