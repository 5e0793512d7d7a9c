"""ctypes binding of libfvna3d.so (include/fvna3d.h): argument marshalling
only.  PyTorch supplies device memory and the stream.  Importing this module
raises if the library is missing: there is no CPU fallback."""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (its HIP runtime first)

from .fvna import BCS, E_NONFINITE, E_NONHYPERBOLIC, E_RETRIES, PRECISION, FvnaError, fvna_stats

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FVNA3D_LIB") or os.path.join(_HERE, "libfvna3d.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it (paper_1311_3004_amd.build3d)")
lib = ctypes.CDLL(LIB_PATH)


class fvna3_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("c0", ctypes.c_double), ("rho0", ctypes.c_double),
                ("beta", ctypes.c_double), ("delta", ctypes.c_double), ("precision", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 6), ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double),
                ("max_retries", ctypes.c_int32), ("fixed_dt", ctypes.c_int32), ("dt0", ctypes.c_double)]


_st, _vp, _dp = ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
for _name, _res, _args in [
        ("fvna3_workspace_size", _st, [ctypes.POINTER(fvna3_params), ctypes.POINTER(ctypes.c_size_t),
                                       ctypes.POINTER(ctypes.c_size_t)]),
        ("fvna3_create", _st, [ctypes.POINTER(fvna3_params), _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
        ("fvna3_set_state", _st, [_vp, _dp, _dp, _dp, _dp]),
        ("fvna3_step", _st, [_vp, ctypes.c_int64]),
        ("fvna3_get_state", _st, [_vp, _dp, _dp, _dp, _dp]),
        ("fvna3_get_stats", _st, [_vp, ctypes.POINTER(fvna_stats)]),
        ("fvna3_time_step_kernels", _st, [_vp, ctypes.c_int32, _dp]),
        ("fvna3_last_error", ctypes.c_char_p, []),
        ("fvna3_destroy", None, [_vp])]:
    _f = getattr(lib, _name)
    _f.restype, _f.argtypes = _res, _args

EXPORTS = ["fvna3_workspace_size", "fvna3_create", "fvna3_set_state", "fvna3_step", "fvna3_get_state",
           "fvna3_get_stats", "fvna3_time_step_kernels", "fvna3_last_error", "fvna3_destroy"]


def check(status, allow=()):
    if status != 0 and status not in allow:
        raise FvnaError(status, lib.fvna3_last_error().decode())
    return status


def make_params(nx, ny, nz, dx, medium, bc=("extrap0",) * 6, precision="f64", cfl_target=0.9, cfl_max=1.0,
                max_retries=8, fixed_dt=False, dt0=0.0):
    p = fvna3_params()
    p.nx, p.ny, p.nz, p.dx = int(nx), int(ny), int(nz), float(dx)
    p.c0, p.rho0 = float(medium["c0"]), float(medium["rho0"])
    p.beta, p.delta = float(medium["beta"]), float(medium["delta"])
    p.precision = PRECISION[precision]
    for k, b in enumerate(bc):
        p.bc[k] = BCS[b]
    p.cfl_target, p.cfl_max, p.max_retries = float(cfl_target), float(cfl_max), int(max_retries)
    p.fixed_dt, p.dt0 = int(bool(fixed_dt)), float(dt0)
    return p


def _dptr(a):
    return a.ctypes.data_as(_dp)


class Sim3:
    """One 3-D simulation: its torch device buffers and an fvna3_ctx."""

    def __init__(self, params, device="cuda:0"):
        import torch
        self.params = params
        sb, xb = ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.fvna3_workspace_size(ctypes.byref(params), ctypes.byref(sb), ctypes.byref(xb)))
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.bufs = [torch.empty(sb.value, dtype=torch.uint8, device=self.device) for _ in range(3)]
            self.scratch = torch.empty(xb.value, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
        h = _vp()
        check(lib.fvna3_create(ctypes.byref(params), *[b.data_ptr() for b in self.bufs], self.scratch.data_ptr(),
                               self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h

    @property
    def shape(self):
        return (self.params.nz, self.params.ny, self.params.nx)

    def fvna3_set_state(self, rho_p, m1, m2, m3):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho_p, m1, m2, m3)]
        for a in arrs:
            assert a.shape == self.shape
        check(lib.fvna3_set_state(self.handle, *[_dptr(a) for a in arrs]))

    def fvna3_step(self, nsteps, allow_device_errors=False):
        allow = (E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES) if allow_device_errors else ()
        return check(lib.fvna3_step(self.handle, int(nsteps)), allow)

    def fvna3_get_state(self):
        out = [np.empty(self.shape, dtype=np.float64) for _ in range(4)]
        check(lib.fvna3_get_state(self.handle, *[_dptr(a) for a in out]))
        return tuple(out)

    def fvna3_get_stats(self):
        s = fvna_stats()
        check(lib.fvna3_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in fvna_stats._fields_}

    def fvna3_time_step_kernels(self, reps):
        ms = ctypes.c_double()
        check(lib.fvna3_time_step_kernels(self.handle, int(reps), ctypes.byref(ms)))
        return ms.value

    def fvna3_destroy(self):
        if self.handle:
            lib.fvna3_destroy(self.handle)
            self.handle = None
