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
    (dict(Lx=4, Ly=4, cx=2, cy=2, d=3, model=1, h=1.0), -1),   # the Ising model needs d = 2
    (dict(Lx=4, Ly=4, cx=2, cy=2, h=0.5), -1),                 # h only for the Ising model
    (dict(Lx=4, Ly=4, cx=2, cy=2, model=2), -1),
    (dict(Lx=4, Ly=1, cx=2, cy=1, d=2, periodic=False, model=1, init_state=2), -2),
    (dict(Lx=4, Ly=4, cx=2, cy=2, gamma_loss=-0.1), -1),                      # negative rate
    (dict(Lx=4, Ly=4, cx=2, cy=2, gamma_deph=float("nan")), -1),
    (dict(Lx=4, Ly=4, cx=2, cy=2, d=2, model=1, h=1.0, gamma_deph=0.1), -2),   # spin model: closed only
    (dict(Lx=4, Ly=4, cx=2, cy=2, d=4, layout=2), -1),                        # no such layout
    (dict(Lx=4, Ly=4, cx=2, cy=2, d=3, layout=1), -2),                        # packed: D = 256 only
    (dict(Lx=4, Ly=4, cx=2, cy=1, d=4, layout=1), -2),
])
def test_plan_create_rejects_before_touching_the_device(kw, code):
    lib = cd.library()
    prob = cd.Problem(**kw)
    h = ctypes.c_void_p()
    st = lib.cdtwa_plan_create(ctypes.byref(prob.c()), 4, ctypes.byref(h))
    assert st == code
    assert not h.value
    assert len(lib.cdtwa_last_error()) > 0


@pytest.mark.parametrize("n_traj", [0, -3])
def test_plan_create_rejects_empty_batches(n_traj):
    lib = cd.library()
    h = ctypes.c_void_p()
    st = lib.cdtwa_plan_create(ctypes.byref(cd.Problem(4, 4, 2, 2).c()), n_traj, ctypes.byref(h))
    assert st == -1 and not h.value
    assert b"n_traj" in lib.cdtwa_last_error()


def test_plan_create_rejects_oversized_grids():
    lib = cd.library()
    h = ctypes.c_void_p()
    st = lib.cdtwa_plan_create(ctypes.byref(cd.Problem(32, 32, 2, 2).c()), (1 << 31) // 1024 + 1, ctypes.byref(h))
    assert st == -1 and not h.value
    assert "batches" in lib.cdtwa_last_error().decode()


def test_spin_limit_environment_is_validated(monkeypatch):
    lib = cd.library()
    h = ctypes.c_void_p()
    for bad in ("abc", "-1", "1e3", "99999999999"):
        monkeypatch.setenv("CDTWA_SPIN_LIMIT", bad)
        assert lib.cdtwa_plan_create(ctypes.byref(cd.Problem(4, 4, 2, 2).c()), 2, ctypes.byref(h)) == -1
        assert not h.value and b"CDTWA_SPIN_LIMIT" in lib.cdtwa_last_error()


def test_null_arguments_are_rejected():
    lib = cd.library()
    assert lib.cdtwa_step_rk4(None, None, None, 0.01, 1, None) == -1
    assert lib.cdtwa_step_rk4_compensated(None, None, None, None, 0.01, 1, None) == -1
    assert lib.cdtwa_sample_noise(None, 0, 0, None, None, None) == -1
    assert lib.cdtwa_plan_destroy(None) == -1
    assert lib.cdtwa_status_string(-3) == b"HIP error"


def test_problem_struct_layout_matches_header(tmp_path):
    """The ctypes mirror of cdtwa_problem has the header's size and offsets."""
    import subprocess
    fields = [f[0] for f in cd.binding._CProblem._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"cdtwa.h\"\nint main(void){printf(\"%zu\", sizeof(cdtwa_problem));"
                   + "".join(f'printf(" %zu", offsetof(cdtwa_problem, {f}));' for f in fields) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cd.binding._CProblem) == 80
    assert got[1:] == [getattr(cd.binding._CProblem, f).offset for f in fields]
