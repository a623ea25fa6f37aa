"""cdtwa_step_rk4_noalloc (the RK4 steps with the library's static device
scratch buffer as workspace) against cdtwa_step_rk4 with a caller workspace:
the same kernels, so the states must agree bit for bit.  Two calls in a row
on the shared buffer, the second on a smaller problem; every path that a
small plan can take (fused 27-row FP64 and FP32, per-stage, trajectory-resident,
fused spin); and
a plan whose workspace exceeds the buffer is rejected before anything runs."""
import ctypes
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

cd = pytest.importorskip("paper_2404_18594_amd")


def _say(*a):
    print(*a, flush=True)


def _plan(prob, n, path=None):
    old = os.environ.get("CDTWA_PATH")
    try:
        if path:
            os.environ["CDTWA_PATH"] = path
        else:
            os.environ.pop("CDTWA_PATH", None)
        return cd.Plan(prob, n)
    finally:
        if old is None:
            os.environ.pop("CDTWA_PATH", None)
        else:
            os.environ["CDTWA_PATH"] = old


def _both(prob, n, seed, dt, steps, path=None, expect_path=None):
    p = _plan(prob, n, path)
    if expect_path is not None:
        assert p.path == expect_path, p.path
    a = p.new_state()
    p.sample_noise(seed, 3, a)
    b = a.clone()
    ws = p.new_workspace()
    p.step_rk4(a, ws, dt, steps)
    p.step_rk4_noalloc(b, dt, steps)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(b)).all()
    same = torch.equal(a, b)
    _say(f"  {prob.Lx}x{prob.Ly} {prob.cx}x{prob.cy} d={prob.d} dtype={prob.dtype} path={p.path}: "
         f"bit-equal {same}, max diff {(a - b).abs().max().item():.2e}")
    assert same
    return p


# (first problem, second smaller problem): fused 27-row FP64, FP32, per-stage,
# trajectory-resident, fused spin
CASES = [
    ((cd.Problem(8, 8, 2, 2, d=3, dtype=cd.F64), 5, None, 1), (cd.Problem(4, 4, 2, 2, d=3, dtype=cd.F64), 2, None, 1)),
    ((cd.Problem(8, 8, 2, 2, d=3, dtype=cd.F32), 7, None, 1), (cd.Problem(4, 4, 2, 2, d=3, dtype=cd.F32), 3, None, 1)),
    ((cd.Problem(6, 6, 1, 1, d=3, dtype=cd.F64), 6, "generic", 0),
     (cd.Problem(4, 4, 2, 1, d=3, dtype=cd.F64), 2, "generic", 0)),
    ((cd.Problem(6, 6, 1, 1, d=3, dtype=cd.F64), 6, None, 6), (cd.Problem(4, 4, 2, 1, d=3, dtype=cd.F32), 2, None, 6)),
    ((cd.Problem(8, 8, 2, 2, d=2, J=1.0, U=0.0, model=1, h=1.0, init_state=1, dtype=cd.F64), 4, None, 5),
     (cd.Problem(4, 4, 2, 2, d=2, J=1.0, U=0.0, model=1, h=1.0, init_state=1, dtype=cd.F64), 1, None, 5)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_equals_step_rk4_on_two_calls(first, second):
    _say("step_rk4_noalloc vs step_rk4")
    for i, (prob, n, path, expect) in enumerate((first, second)):
        _both(prob, n, 40 + i, 0.01, 12 - 5 * i, path, expect)


def test_noalloc_rejects_plans_beyond_the_buffer():
    _say("step_rk4_noalloc: oversize plan")
    p = _plan(cd.Problem(32, 32, 2, 2, d=3, dtype=cd.F64), 2, "generic")
    assert p.path == 0
    rho = p.new_state()
    p.sample_noise(1, 0, rho)
    before = rho.clone()
    lib = cd.library()
    st = lib.cdtwa_step_rk4_noalloc(p._h, ctypes.c_void_p(rho.data_ptr()), 0.01, 3,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == -1
    assert b"static scratch buffer" in lib.cdtwa_last_error()
    assert torch.equal(rho, before)
    # and the buffer still works afterwards
    _both(cd.Problem(4, 4, 2, 2, d=3, dtype=cd.F64), 2, 9, 0.01, 4, None, 1)
