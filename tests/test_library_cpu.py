"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/cdtwa.h, and rejects invalid problems
before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2404_18594_amd as cd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "cdtwa.h")).read()
    return sorted(set(re.findall(r"\b(cdtwa_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(cd.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = cd.library()
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("kw,code", [
    (dict(Lx=4, Ly=4, cx=3, cy=2), -1),          # cluster side 3
    (dict(Lx=5, Ly=4, cx=2, cy=2), -1),          # not divisible
    (dict(Lx=2, Ly=4, cx=2, cy=2), -1),          # periodic with one cluster along x
    (dict(Lx=4, Ly=4, cx=2, cy=2, d=5), -1),     # d out of range
    (dict(Lx=4, Ly=4, cx=2, cy=2, init_state=1), -2),
])
def test_plan_create_rejects_before_touching_the_device(kw, code):
    lib = cd.library()
    prob = cd.Problem(**kw)
    h = ctypes.c_void_p()
    st = lib.cdtwa_plan_create(ctypes.byref(prob.c()), 4, ctypes.byref(h))
    assert st == code
    assert not h.value
    assert len(lib.cdtwa_last_error()) > 0


def test_null_arguments_are_rejected():
    lib = cd.library()
    assert lib.cdtwa_step_rk4(None, None, None, 0.01, 1, None) == -1
    assert lib.cdtwa_sample_noise(None, 0, 0, None, None, None) == -1
    assert lib.cdtwa_plan_destroy(None) == -1
    assert lib.cdtwa_status_string(-3) == b"HIP error"
