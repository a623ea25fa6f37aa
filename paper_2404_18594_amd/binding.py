"""Thin ctypes binding of libcdtwa.so (the C ABI in include/cdtwa.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch supplies device memory (complex128 / complex64 tensors
for the state, float64 tensors for observables) and the current HIP stream.
If the library is not built the import of this module still works, but every
call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdtwa.so")

NOBS = 15
OBS_NAMES = [
    "csp_10", "csp_01", "csp_11", "csp_20", "csp_02",
    "nn_10", "nn_01", "nn_11", "nn_20", "nn_02",
    "density", "energy", "purity", "trace_dev", "herm_dev",
]
F32, F64 = 0, 1
LAYOUT_FULL, LAYOUT_PACKED = 0, 1
PACKED_TILE, PACKED_ELEMS = 16, 34816

EXPORTS = [
    "cdtwa_plan_create", "cdtwa_plan_destroy", "cdtwa_plan_info", "cdtwa_workspace_bytes",
    "cdtwa_sample_noise", "cdtwa_gather_boundary_fields", "cdtwa_commutator", "cdtwa_step_rk4",
    "cdtwa_accumulate_observables", "cdtwa_plan_path", "cdtwa_device_status", "cdtwa_step_rk4_schedule",
    "cdtwa_mlp_workspace_bytes", "cdtwa_mlp_init", "cdtwa_mlp_forward", "cdtwa_mlp_backward", "cdtwa_mlp_adam",
    "cdtwa_cv_features", "cdtwa_cv_targets", "cdtwa_cv_traj_sums", "cdtwa_cv_sample_features",
    "cdtwa_cv_workspace_bytes", "cdtwa_cv_expectation",
    "cdtwa_batch_create", "cdtwa_batch_destroy", "cdtwa_batch_workspace_bytes", "cdtwa_batch_step_rk4",
    "cdtwa_batch_info", "cdtwa_step_rk4_noalloc", "cdtwa_step_rk4_compensated",
    "cdtwa_status_string", "cdtwa_last_error",
]
MLP_IN, MLP_HIDDEN, MLP_OUT = 128, 256, 64
MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_OUT + MLP_OUT
MLP_WBF16 = MLP_IN * MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN * MLP_OUT


class CdtwaError(RuntimeError):
    pass


class _CProblem(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32), ("cx", ctypes.c_int32), ("cy", ctypes.c_int32),
                ("d", ctypes.c_int32), ("periodic", ctypes.c_int32), ("J", ctypes.c_double), ("U", ctypes.c_double),
                ("init_state", ctypes.c_int32), ("dtype", ctypes.c_int32), ("model", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("h", ctypes.c_double), ("gamma_deph", ctypes.c_double),
                ("gamma_loss", ctypes.c_double)]


_lib = None


def library():
    """Load libcdtwa.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise CdtwaError(f"{LIB_PATH} is missing: build it with `python paper_2404_18594_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER(_CProblem)
    lib.cdtwa_plan_create.argtypes = [P, i64, ctypes.POINTER(vp)]
    lib.cdtwa_plan_destroy.argtypes = [vp]
    lib.cdtwa_plan_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 6
    lib.cdtwa_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.cdtwa_sample_noise.argtypes = [vp, ctypes.c_uint64, i64, vp, vp, vp]
    lib.cdtwa_gather_boundary_fields.argtypes = [vp, vp, vp, vp, vp]
    lib.cdtwa_commutator.argtypes = [vp, vp, vp, vp, vp]
    lib.cdtwa_step_rk4.argtypes = [vp, vp, vp, ctypes.c_double, i32, vp]
    lib.cdtwa_step_rk4_schedule.argtypes = [vp, vp, vp, ctypes.c_double, i32, vp, vp, vp]
    lib.cdtwa_step_rk4_noalloc.argtypes = [vp, vp, ctypes.c_double, i32, vp]
    lib.cdtwa_step_rk4_compensated.argtypes = [vp, vp, vp, vp, ctypes.c_double, i32, vp]
    lib.cdtwa_accumulate_observables.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.cdtwa_plan_path.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.cdtwa_device_status.argtypes = [vp, vp, ctypes.POINTER(i32), vp]
    sz = ctypes.POINTER(ctypes.c_size_t)
    u64, f32 = ctypes.c_uint64, ctypes.c_float
    lib.cdtwa_mlp_workspace_bytes.argtypes = [i64, sz]
    lib.cdtwa_mlp_init.argtypes = [vp, vp, u64, vp]
    lib.cdtwa_mlp_forward.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    lib.cdtwa_mlp_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp]
    lib.cdtwa_mlp_adam.argtypes = [vp, vp, vp, vp, vp, f32, i32, vp]
    lib.cdtwa_cv_features.argtypes = [vp, vp, vp, vp]
    lib.cdtwa_cv_targets.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.cdtwa_cv_traj_sums.argtypes = [vp, vp, vp, vp]
    lib.cdtwa_cv_sample_features.argtypes = [vp, u64, i64, i64, vp, vp]
    lib.cdtwa_cv_workspace_bytes.argtypes = [sz]
    lib.cdtwa_cv_expectation.argtypes = [vp, vp, vp, u64, i64, vp, vp, vp]
    lib.cdtwa_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
    lib.cdtwa_batch_destroy.argtypes = [vp]
    lib.cdtwa_batch_workspace_bytes.argtypes = [vp, i32, sz]
    lib.cdtwa_batch_step_rk4.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double, i32, vp]
    lib.cdtwa_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                     ctypes.POINTER(i32), ctypes.POINTER(i32)]
    for f in EXPORTS[:-2]:
        getattr(lib, f).restype = ctypes.c_int
    lib.cdtwa_status_string.argtypes = [ctypes.c_int]
    lib.cdtwa_status_string.restype = ctypes.c_char_p
    lib.cdtwa_last_error.argtypes = []
    lib.cdtwa_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st != 0:
        lib = library()
        raise CdtwaError(f"{what}: {lib.cdtwa_status_string(st).decode()} ({lib.cdtwa_last_error().decode()})")


@dataclass(frozen=True)
class Problem:
    """Lattice Lx x Ly cut into cx x cy clusters, local dimension d; dtype F64
    or F32 trajectory state.  model 0: Bose-Hubbard (arXiv:2404.18594 Sec. III
    Eq. (H_bose)), init_state 0 = Mott |1>.  model 1 (d = 2): transverse-field
    Ising J s^z s^z + h s^x (App. A Eq. (Hising)), init_state 0 = all up,
    1 = Neel.  gamma_deph, gamma_loss (model 0): local Lindblad rates of
    L = n_j and L = a_j on every cluster matrix.  layout: LAYOUT_FULL, or
    LAYOUT_PACKED (2x2 clusters with d = 4: the upper 16x16 tiles only)."""
    Lx: int
    Ly: int
    cx: int
    cy: int
    d: int = 3
    periodic: bool = True
    J: float = 1.0
    U: float = 5.0
    dtype: int = F64
    init_state: int = 0
    model: int = 0
    h: float = 0.0
    gamma_deph: float = 0.0
    gamma_loss: float = 0.0
    layout: int = LAYOUT_FULL

    def c(self) -> _CProblem:
        return _CProblem(self.Lx, self.Ly, self.cx, self.cy, self.d, int(self.periodic), self.J, self.U,
                         self.init_state, self.dtype, self.model, int(self.layout), self.h, self.gamma_deph,
                         self.gamma_loss)

    @property
    def complex_dtype(self):
        return torch.complex128 if self.dtype == F64 else torch.complex64


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """Owns a cdtwa_plan (geometry and sampling tables on the device)."""

    def __init__(self, problem: Problem, n_traj: int):
        lib = library()
        self.problem = problem
        self.n_traj = int(n_traj)
        h = ctypes.c_void_p()
        _check(lib.cdtwa_plan_create(ctypes.byref(problem.c()), self.n_traj, ctypes.byref(h)), "plan_create")
        self._h = h
        vals = [ctypes.c_int32() for _ in range(6)]
        _check(lib.cdtwa_plan_info(self._h, *[ctypes.byref(v) for v in vals]), "plan_info")
        self.n_sites, self.n_clusters, self.n_local, self.D, self.n_gen, self.real_bytes = [v.value for v in vals]
        nb = ctypes.c_size_t()
        _check(lib.cdtwa_workspace_bytes(self._h, ctypes.byref(nb)), "workspace_bytes")
        self.workspace_bytes = nb.value
        path, res = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.cdtwa_plan_path(self._h, ctypes.byref(path), ctypes.byref(res)), "plan_path")
        self.path, self.resident = path.value, res.value

    def device_status(self, ws, stream=None) -> int:
        """Synchronises and returns the status word of the last step_rk4."""
        st = ctypes.c_int32()
        _check(library().cdtwa_device_status(self._h, _ptr(ws), ctypes.byref(st), _stream(stream)), "device_status")
        return st.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().cdtwa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers -------------------------------------------------------
    def state_shape(self):
        if self.problem.layout == LAYOUT_PACKED:
            return (self.n_traj, self.n_clusters, PACKED_ELEMS)
        return (self.n_traj, self.n_clusters, self.D, self.D)

    def new_state(self, device="cuda"):
        return torch.empty(self.state_shape(), dtype=self.problem.complex_dtype, device=device)

    def new_workspace(self, device="cuda"):
        return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)

    def _chk_state(self, t, name):
        if t.dtype != self.problem.complex_dtype or not t.is_contiguous() or tuple(t.shape) != self.state_shape():
            raise CdtwaError(f"{name}: expected contiguous {self.problem.complex_dtype} {self.state_shape()}")
        if not t.is_cuda:
            raise CdtwaError(f"{name}: must be a device tensor")

    def _chk_ws(self, ws):
        if ws.numel() * ws.element_size() < self.workspace_bytes or not ws.is_cuda:
            raise CdtwaError("workspace too small")

    # ---- C ABI ---------------------------------------------------------
    def sample_noise(self, seed: int, traj_offset: int, rho, noise=None, stream=None):
        self._chk_state(rho, "rho")
        if noise is not None:
            if noise.dtype != torch.int8 or tuple(noise.shape) != (self.n_traj, self.n_sites, self.n_gen) \
                    or not noise.is_contiguous():
                raise CdtwaError("noise: expected contiguous int8 [n_traj][Ns][n_gen]")
        _check(library().cdtwa_sample_noise(self._h, int(seed), int(traj_offset), _ptr(noise), _ptr(rho),
                                            _stream(stream)), "sample_noise")

    def gather_boundary_fields(self, rho, b, phi, stream=None):
        self._chk_state(rho, "rho")
        shape = (self.n_traj, self.n_sites)
        for t in (b, phi):
            if tuple(t.shape) != shape or t.dtype != self.problem.complex_dtype or not t.is_contiguous():
                raise CdtwaError("b/phi: expected contiguous complex [n_traj][Ns]")
        _check(library().cdtwa_gather_boundary_fields(self._h, _ptr(rho), _ptr(b), _ptr(phi), _stream(stream)),
               "gather_boundary_fields")

    def commutator(self, rho, K, ws, stream=None):
        self._chk_state(rho, "rho")
        self._chk_state(K, "K")
        self._chk_ws(ws)
        _check(library().cdtwa_commutator(self._h, _ptr(rho), _ptr(K), _ptr(ws), _stream(stream)), "commutator")

    def step_rk4(self, rho, ws, dt: float, n_steps: int, stream=None):
        self._chk_state(rho, "rho")
        self._chk_ws(ws)
        _check(library().cdtwa_step_rk4(self._h, _ptr(rho), _ptr(ws), float(dt), int(n_steps), _stream(stream)),
               "step_rk4")

    def step_rk4_noalloc(self, rho, dt: float, n_steps: int, stream=None):
        """step_rk4 with the library's static device scratch buffer as its
        workspace (no allocation; calls on one device must not overlap)."""
        self._chk_state(rho, "rho")
        _check(library().cdtwa_step_rk4_noalloc(self._h, _ptr(rho), float(dt), int(n_steps), _stream(stream)),
               "step_rk4_noalloc")

    def low_parts_shape(self):
        return (self.n_traj, self.n_clusters, PACKED_ELEMS)

    def new_low_parts(self, device="cuda"):
        """Zero low parts for step_rk4_compensated (exact for a state fresh
        from sample_noise): FP32 complex [n_traj][n_clusters][PACKED_ELEMS]."""
        return torch.zeros(self.low_parts_shape(), dtype=torch.complex64, device=device)

    def step_rk4_compensated(self, rho, rho_lo, ws, dt: float, n_steps: int, stream=None):
        """step_rk4 on the FP32 state rho + rho_lo (rho_lo: the packed FP32
        low parts, updated in place); FP32 plans with 2x2 clusters, d = 4."""
        self._chk_state(rho, "rho")
        if rho_lo.dtype != torch.complex64 or not rho_lo.is_contiguous() or not rho_lo.is_cuda \
                or tuple(rho_lo.shape) != self.low_parts_shape():
            raise CdtwaError(f"rho_lo: expected contiguous device complex64 {self.low_parts_shape()}")
        self._chk_ws(ws)
        _check(library().cdtwa_step_rk4_compensated(self._h, _ptr(rho), _ptr(rho_lo), _ptr(ws), float(dt),
                                                    int(n_steps), _stream(stream)), "step_rk4_compensated")

    def step_rk4_schedule(self, rho, ws, dt: float, n_steps: int, c1_half, c2_half, stream=None):
        """RK4 with the couplings (J, U) -- (J, h) for the Ising model -- at
        every half step: sequences of 2*n_steps+1 floats (host)."""
        self._chk_state(rho, "rho")
        self._chk_ws(ws)
        c1 = (ctypes.c_double * len(c1_half))(*[float(v) for v in c1_half])
        c2 = (ctypes.c_double * len(c2_half))(*[float(v) for v in c2_half])
        if len(c1) != 2 * int(n_steps) + 1 or len(c2) != len(c1):
            raise CdtwaError("schedules need 2*n_steps+1 half-step values")
        _check(library().cdtwa_step_rk4_schedule(self._h, _ptr(rho), _ptr(ws), float(dt), int(n_steps), c1, c2,
                                                 _stream(stream)), "step_rk4_schedule")

    def accumulate_observables(self, rho, t_index: int, sums, ws, per_traj=None, stream=None):
        self._chk_state(rho, "rho")
        self._chk_ws(ws)
        if sums.dtype != torch.float64 or not sums.is_contiguous() or sums.numel() < (t_index + 1) * NOBS * 3:
            raise CdtwaError("sums: expected contiguous float64 [n_times][NOBS][3]")
        if per_traj is not None and (per_traj.dtype != torch.float64 or tuple(per_traj.shape) != (self.n_traj, NOBS)
                                     or not per_traj.is_contiguous()):
            raise CdtwaError("per_traj: expected contiguous float64 [n_traj][NOBS]")
        _check(library().cdtwa_accumulate_observables(self._h, _ptr(rho), int(t_index), _ptr(sums), _ptr(per_traj),
                                                      _ptr(ws), _stream(stream)), "accumulate_observables")

    # ---- control variate (2x2 clusters, d = 3) -------------------------
    def _chk(self, t, dtype, shape, name):
        if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
            raise CdtwaError(f"{name}: expected contiguous device {dtype} {tuple(shape)}")

    def cv_features(self, noise, features, stream=None):
        self._chk(noise, torch.int8, (self.n_traj, self.n_sites, self.n_gen), "noise")
        self._chk(features, torch.float32, (self.n_traj * self.n_clusters, MLP_IN), "features")
        _check(library().cdtwa_cv_features(self._h, _ptr(noise), _ptr(features), _stream(stream)), "cv_features")

    def cv_targets(self, rho, column: int, targets, ws, stream=None):
        self._chk_state(rho, "rho")
        self._chk_ws(ws)
        self._chk(targets, torch.float32, (self.n_traj * self.n_clusters, MLP_OUT), "targets")
        _check(library().cdtwa_cv_targets(self._h, _ptr(rho), int(column), _ptr(targets), _ptr(ws), _stream(stream)),
               "cv_targets")

    def cv_traj_sums(self, y, gtraj, stream=None):
        self._chk(y, torch.float32, (self.n_traj * self.n_clusters, MLP_OUT), "y")
        self._chk(gtraj, torch.float64, (self.n_traj, MLP_OUT), "gtraj")
        _check(library().cdtwa_cv_traj_sums(self._h, _ptr(y), _ptr(gtraj), _stream(stream)), "cv_traj_sums")

    def cv_sample_features(self, seed: int, first: int, features, stream=None):
        if features.dtype != torch.float32 or features.dim() != 2 or features.shape[1] != MLP_IN \
                or not features.is_contiguous() or not features.is_cuda:
            raise CdtwaError("features: expected contiguous device float32 [n][128]")
        _check(library().cdtwa_cv_sample_features(self._h, int(seed), int(first), features.shape[0], _ptr(features),
                                                  _stream(stream)), "cv_sample_features")

    def cv_expectation(self, mlp, seed: int, n_samples: int, moments, ws=None, stream=None):
        """Adds the moments of g over n_samples i.i.d. patches into moments
        [64][3]; ws: a cv workspace (allocated here when None)."""
        self._chk(moments, torch.float64, (MLP_OUT, 3), "moments")
        if ws is None:
            ws = new_cv_workspace()
        if ws.numel() * ws.element_size() < cv_workspace_bytes() or not ws.is_cuda:
            raise CdtwaError("cv workspace too small")
        _check(library().cdtwa_cv_expectation(self._h, _ptr(mlp.params), _ptr(mlp.wbf16), int(seed), int(n_samples),
                                              _ptr(moments), _ptr(ws), _stream(stream)), "cv_expectation")


def cv_workspace_bytes() -> int:
    nb = ctypes.c_size_t()
    _check(library().cdtwa_cv_workspace_bytes(ctypes.byref(nb)), "cv_workspace_bytes")
    return nb.value


def new_cv_workspace(device="cuda"):
    return torch.empty(cv_workspace_bytes(), dtype=torch.uint8, device=device)


class Mlp:
    """Parameters, BF16 weight copy and Adam moments of the control-variate
    network (device tensors), with the C-ABI calls that act on them."""

    def __init__(self, seed: int = 0, device="cuda", stream=None):
        self.params = torch.empty(MLP_PARAMS, dtype=torch.float32, device=device)
        self.wbf16 = torch.empty(MLP_WBF16, dtype=torch.int16, device=device)
        self.m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=device)
        self.grad = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=device)
        self.step = 0
        _check(library().cdtwa_mlp_init(_ptr(self.params), _ptr(self.wbf16), int(seed), _stream(stream)), "mlp_init")

    def load(self, params, wbf16):
        """Replace the weights (FP32 params and their BF16 bit patterns)."""
        self.params.copy_(params)
        self.wbf16.copy_(wbf16)

    @staticmethod
    def workspace_bytes(n: int) -> int:
        nb = ctypes.c_size_t()
        _check(library().cdtwa_mlp_workspace_bytes(int(n), ctypes.byref(nb)), "mlp_workspace_bytes")
        return nb.value

    @staticmethod
    def new_workspace(n: int, device="cuda"):
        return torch.empty(Mlp.workspace_bytes(n), dtype=torch.uint8, device=device)

    def _rows(self, t, cols, name):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous() or not t.is_cuda:
            raise CdtwaError(f"{name}: expected contiguous device float32 [n][{cols}]")
        return t.shape[0]

    def forward(self, x, y, ws, stream=None):
        n = self._rows(x, MLP_IN, "x")
        if self._rows(y, MLP_OUT, "y") != n:
            raise CdtwaError("x and y row counts differ")
        if ws.numel() < Mlp.workspace_bytes(n):
            raise CdtwaError("mlp workspace too small")
        _check(library().cdtwa_mlp_forward(_ptr(self.params), _ptr(self.wbf16), _ptr(x), _ptr(y), n, _ptr(ws),
                                           _stream(stream)), "mlp_forward")

    def backward(self, y, target, ws, loss=None, stream=None):
        n = self._rows(y, MLP_OUT, "y")
        if self._rows(target, MLP_OUT, "target") != n:
            raise CdtwaError("y and target row counts differ")
        if ws.numel() < Mlp.workspace_bytes(n):
            raise CdtwaError("mlp workspace too small")
        _check(library().cdtwa_mlp_backward(_ptr(self.wbf16), _ptr(y), _ptr(target), _ptr(self.grad), _ptr(loss), n,
                                            _ptr(ws), _stream(stream)), "mlp_backward")

    def adam(self, lr: float, stream=None):
        self.step += 1
        _check(library().cdtwa_mlp_adam(_ptr(self.params), _ptr(self.wbf16), _ptr(self.grad), _ptr(self.m),
                                        _ptr(self.v), float(lr), self.step, _stream(stream)), "mlp_adam")


class Batch:
    """Several plans advanced together (cdtwa_batch_*): one launch per RK4
    stage for every member with d = 3 whose clusters the mixed kernel takes,
    the step captured in a HIP graph; the plans must stay alive."""

    def __init__(self, plans, mix_all: bool = False):
        lib = library()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.cdtwa_batch_create(arr, len(self.plans), 1 if mix_all else 0, ctypes.byref(h)), "batch_create")
        self._h = h

    def workspace_bytes(self, member: int) -> int:
        nb = ctypes.c_size_t()
        _check(library().cdtwa_batch_workspace_bytes(self._h, int(member), ctypes.byref(nb)), "batch_workspace_bytes")
        return nb.value

    def new_workspaces(self, device="cuda"):
        return [torch.empty(max(self.workspace_bytes(i), 1), dtype=torch.uint8, device=device)
                for i in range(len(self.plans))]

    def step_rk4(self, rhos, workspaces, dt: float, n_steps: int, stream=None):
        if len(rhos) != len(self.plans) or len(workspaces) != len(self.plans):
            raise CdtwaError("one state and one workspace per member")
        for i, (p, r, w) in enumerate(zip(self.plans, rhos, workspaces)):
            p._chk_state(r, f"rho[{i}]")
            if w.numel() * w.element_size() < self.workspace_bytes(i) or not w.is_cuda:
                raise CdtwaError(f"workspace[{i}] too small")
        n = len(self.plans)
        ra = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhos])
        wa = (ctypes.c_void_p * n)(*[w.data_ptr() for w in workspaces])
        _check(library().cdtwa_batch_step_rk4(self._h, ra, wa, float(dt), int(n_steps), _stream(stream)),
               "batch_step_rk4")

    def info(self):
        nm, nt, wg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        nr, ri = ctypes.c_int32(), ctypes.c_int64()
        nf, fw = ctypes.c_int32(), ctypes.c_int32()
        var = (ctypes.c_int32 * 3)()
        _check(library().cdtwa_batch_info(self._h, ctypes.byref(nm), ctypes.byref(nt), var, ctypes.byref(wg),
                                          ctypes.byref(nr), ctypes.byref(ri), ctypes.byref(nf), ctypes.byref(fw)),
               "batch_info")
        return {"mixed_members": nm.value, "threads": nt.value, "variants": list(var), "workgroups": wg.value,
                "resident_members": nr.value, "resident_items": ri.value, "fused_members": nf.value,
                "fused_workgroups": fw.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().cdtwa_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
