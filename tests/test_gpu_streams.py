"""The stream argument of the C ABI: sampling, RK4 steps (fused and
per-stage paths, with and without dissipation) and observables enqueued on a
second stream (default priority) give the same bits as on the current
stream, with the buffers allocated on that stream and only that stream
synchronised before the results are read."""
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _plan(prob, n, path):
    old = os.environ.get("CDTWA_PATH")
    os.environ["CDTWA_PATH"] = path
    try:
        return cd.Plan(prob, n)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


def _run(plan, stream):
    with torch.cuda.stream(stream):
        rho, ws = plan.new_state(), plan.new_workspace()
        sums = torch.zeros(2, cd.NOBS, 3, dtype=torch.float64, device="cuda")
        per = torch.zeros(plan.n_traj, cd.NOBS, dtype=torch.float64, device="cuda")
    plan.sample_noise(31, 5, rho, stream=stream)
    plan.accumulate_observables(rho, 0, sums, ws, stream=stream)
    plan.step_rk4(rho, ws, 0.02, 7, stream=stream)
    plan.accumulate_observables(rho, 1, sums, ws, per_traj=per, stream=stream)
    stream.synchronize()
    return rho.cpu(), sums.cpu(), per.cpu()


@pytest.mark.parametrize("path,expect", [("fused27", 1), ("generic", 0)])
@pytest.mark.parametrize("gammas", [(0.0, 0.0), (0.2, 0.1)])
def test_side_stream_matches_current_stream(path, expect, gammas):
    prob = cd.Problem(4, 4, 2, 2, d=3, periodic=True, J=1.0, U=5.0, dtype=cd.F64,
                      gamma_deph=gammas[0], gamma_loss=gammas[1])
    plan = _plan(prob, 5, path)
    assert plan.path == expect
    a = _run(plan, torch.cuda.current_stream())
    side = torch.cuda.Stream()
    b = _run(plan, side)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
