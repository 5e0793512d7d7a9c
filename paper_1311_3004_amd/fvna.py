"""ctypes binding of libfvna (include/fvna.h): the same entry points, same names.

Only argument marshalling happens here: every step of the method runs in the
HIP kernels of libfvna.  PyTorch is used for device memory (tensors whose data
pointers are handed to the library) and for the HIP stream.  There is no
fallback: if libfvna.so is missing or cannot be loaded, importing this module
raises.
"""
import ctypes
import os

import numpy as np
# torch first: its HIP runtime must be the one libfvna binds to (a library
# loaded before torch would pull in a second HIP runtime, whose streams and
# context torch cannot share)
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FVNA_LIB") or os.path.join(_HERE, "libfvna.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES, E_STATE = range(8)
CARTESIAN, AXISYMMETRIC = 0, 1
F64, F32, F32_F16STORE, F32_BF16STORE = 0, 1, 2, 3
BC_PERIODIC, BC_EXTRAP0, BC_REFLECT, BC_TAYLOR, BC_SOURCE = 0, 1, 2, 3, 4

PRECISION = {"f64": F64, "f32": F32, "f32_f16store": F32_F16STORE, "f32_bf16store": F32_BF16STORE}
GEOMETRY = {"planar": CARTESIAN, "cartesian": CARTESIAN, "axisym": AXISYMMETRIC}
BCS = {"periodic": BC_PERIODIC, "extrap0": BC_EXTRAP0, "reflect": BC_REFLECT,
       "taylor": BC_TAYLOR, "source": BC_SOURCE}

EXPORTS = [
    "fvna_workspace_size", "fvna_create", "fvna_set_bc", "fvna_set_source", "fvna_set_taylor",
    "fvna_set_state", "fvna_set_clock", "fvna_step", "fvna_sync", "fvna_shift", "fvna_step_window",
    "fvna_set_recorder",
    "fvna_get_state", "fvna_get_window",
    "fvna_get_stats", "fvna_sums", "fvna_sums_noalloc", "fvna_taylor_errors", "fvna_time_step_kernel", "fvna_autotune", "fvna_get_tile_rows",
    "fvna_last_error", "fvna_destroy", "fvna_batch_create", "fvna_batch_set_state",
    "fvna_batch_step", "fvna_batch_sync", "fvna_batch_get_state", "fvna_batch_get_stats",
    "fvna_batch_time_step_kernel", "fvna_batch_autotune", "fvna_batch_get_tile_rows", "fvna_batch_destroy",
]


class fvna_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double),
        ("c0", ctypes.c_double), ("rho0", ctypes.c_double), ("beta", ctypes.c_double),
        ("delta", ctypes.c_double), ("geometry", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4), ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double),
        ("max_retries", ctypes.c_int32), ("dt0", ctypes.c_double), ("fixed_dt", ctypes.c_int32),
        ("store_scale", ctypes.c_double * 3), ("tile_rows", ctypes.c_int32),
    ]


class fvna_source(ctypes.Structure):
    _fields_ = [("freq", ctypes.c_double), ("p_surface", ctypes.c_double),
                ("focal_length", ctypes.c_double), ("aperture", ctypes.c_double),
                ("ramp_cycles", ctypes.c_double), ("envelope", ctypes.c_int32),
                ("packet_cycles", ctypes.c_double), ("second_stage", ctypes.c_int32),
                ("stage2_time", ctypes.c_double)]


ENVELOPES = {"ramp": 0, "packet": 1}


class fvna_window(ctypes.Structure):
    _fields_ = [("t1", ctypes.c_double), ("check_every", ctypes.c_int32), ("quantum", ctypes.c_int32),
                ("speed", ctypes.c_double)]


class fvna_window_state(ctypes.Structure):
    _fields_ = [("x_off", ctypes.c_int64), ("phase", ctypes.c_int64)]


class fvna_recorder(ctypes.Structure):
    _fields_ = [("row", ctypes.c_int32), ("probe_col", ctypes.c_int32), ("path_len", ctypes.c_int64),
                ("row_max", ctypes.c_void_p), ("probe_t", ctypes.c_void_p), ("probe_rho", ctypes.c_void_p),
                ("capacity", ctypes.c_int64)]


class fvna_stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_next", ctypes.c_double), ("nu_last", ctypes.c_double),
                ("nu_mean", ctypes.c_double), ("nu_std", ctypes.c_double),
                ("steps", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("status", ctypes.c_int32), ("status_step", ctypes.c_int64)]


class FvnaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfvna status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfvna.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, st, i32, i64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "fvna_workspace_size": (st, [P(fvna_params), P(ctypes.c_size_t), P(ctypes.c_size_t)]),
        "fvna_create": (st, [P(fvna_params), vp, vp, vp, vp, P(vp)]),
        "fvna_set_bc": (st, [vp, i32, i32]),
        "fvna_set_source": (st, [vp, i32, P(fvna_source)]),
        "fvna_set_taylor": (st, [vp, d, d, d]),
        "fvna_set_state": (st, [vp, dp, dp, dp]),
        "fvna_set_clock": (st, [vp, d, d]),
        "fvna_step": (st, [vp, i64]),
        "fvna_sync": (st, [vp]),
        "fvna_shift": (st, [vp, i32]),
        "fvna_step_window": (st, [vp, P(fvna_window), P(fvna_window_state), i64]),
        "fvna_set_recorder": (st, [vp, P(fvna_recorder)]),
        "fvna_get_state": (st, [vp, dp, dp, dp]),
        "fvna_get_window": (st, [vp, i32, i32, i32, i32, dp, dp, dp]),
        "fvna_get_stats": (st, [vp, P(fvna_stats)]),
        "fvna_sums": (st, [vp, dp]),
        "fvna_sums_noalloc": (st, [P(fvna_params), vp, vp, vp]),
        "fvna_taylor_errors": (st, [vp, d, d, d, dp]),
        "fvna_time_step_kernel": (st, [vp, i32, dp]),
        "fvna_autotune": (st, [vp, P(i32)]),
        "fvna_get_tile_rows": (st, [vp, P(i32)]),
        "fvna_last_error": (ctypes.c_char_p, []),
        "fvna_destroy": (None, [vp]),
        "fvna_batch_create": (st, [i32, P(fvna_params), P(vp), vp, P(vp)]),
        "fvna_batch_set_state": (st, [vp, i32, dp, dp, dp]),
        "fvna_batch_step": (st, [vp, i64]),
        "fvna_batch_sync": (st, [vp]),
        "fvna_batch_get_state": (st, [vp, i32, dp, dp, dp]),
        "fvna_batch_get_stats": (st, [vp, i32, P(fvna_stats)]),
        "fvna_batch_time_step_kernel": (st, [vp, i32, dp]),
        "fvna_batch_autotune": (st, [vp, P(i32)]),
        "fvna_batch_get_tile_rows": (st, [vp, P(i32)]),
        "fvna_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def last_error():
    return lib.fvna_last_error().decode()


def check(status, allow=()):
    if status != OK and status not in allow:
        raise FvnaError(status, last_error())
    return status


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, dx, medium, bc=("extrap0",) * 4, geometry="planar", precision="f32",
                cfl_target=0.9, cfl_max=1.0, max_retries=8, dt0=0.0, fixed_dt=False,
                store_scale=(0.0, 0.0, 0.0), tile_rows=0):
    p = fvna_params()
    p.nx, p.ny, p.dx = int(nx), int(ny), float(dx)
    p.c0, p.rho0 = float(medium["c0"]), float(medium["rho0"])
    p.beta, p.delta = float(medium["beta"]), float(medium["delta"])
    p.geometry = GEOMETRY[geometry] if isinstance(geometry, str) else int(geometry)
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    for k, b in enumerate(bc):
        p.bc[k] = BCS[b] if isinstance(b, str) else int(b)
    p.cfl_target, p.cfl_max = float(cfl_target), float(cfl_max)
    p.max_retries, p.dt0, p.fixed_dt = int(max_retries), float(dt0), int(bool(fixed_dt))
    for k in range(3):
        p.store_scale[k] = float(store_scale[k])
    p.tile_rows = int(tile_rows)
    return p


def workspace_size(p):
    sb, xb = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib.fvna_workspace_size(ctypes.byref(p), ctypes.byref(sb), ctypes.byref(xb)))
    return sb.value, xb.value


def _device_buffer(nbytes, device):
    import torch
    # uint8 tensors from the caching allocator are 512-byte aligned
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Sim:
    """One simulation: owns its torch device buffers and an fvna_ctx."""

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        self.params = params
        self.device = torch.device(device)
        sb, xb = workspace_size(params)
        with torch.cuda.device(self.device):
            self.buf_a = _device_buffer(sb, self.device)
            self.buf_b = _device_buffer(sb, self.device)
            self.scratch = _device_buffer(xb, self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(lib.fvna_create(ctypes.byref(params), ctypes.c_void_p(self.buf_a.data_ptr()),
                                  ctypes.c_void_p(self.buf_b.data_ptr()),
                                  ctypes.c_void_p(self.scratch.data_ptr()),
                                  _stream_handle(self.stream), ctypes.byref(h)))
        self.handle = h

    @property
    def shape(self):
        return (self.params.ny, self.params.nx)

    # --- the C entry points, one to one ---
    def fvna_set_bc(self, side, bc):
        check(lib.fvna_set_bc(self.handle, int(side), BCS[bc] if isinstance(bc, str) else int(bc)))

    def fvna_set_source(self, side, freq, p_surface, focal_length, aperture, ramp_cycles=3.0,
                        envelope="ramp", packet_cycles=4.0, stage2_time=None):
        """stage2_time None: the source stays on; else the time [s] from which
        the whole side is zero-order extrapolation."""
        env = ENVELOPES[envelope] if isinstance(envelope, str) else int(envelope)
        s = fvna_source(float(freq), float(p_surface), float(focal_length), float(aperture),
                        float(ramp_cycles), env, float(packet_cycles), int(stage2_time is not None),
                        float(stage2_time) if stage2_time is not None else 0.0)
        check(lib.fvna_set_source(self.handle, int(side), ctypes.byref(s)))

    def fvna_set_taylor(self, amplitude_pa, x0_m, angle=0.0):
        check(lib.fvna_set_taylor(self.handle, float(amplitude_pa), float(x0_m), float(angle)))

    def fvna_set_state(self, rho_p, mom_x, mom_y):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho_p, mom_x, mom_y)]
        for a in arrs:
            if a.shape != self.shape:
                raise ValueError(f"state arrays must have shape {self.shape}")
        check(lib.fvna_set_state(self.handle, *[_dptr(a) for a in arrs]))

    def fvna_set_clock(self, t, dt_next=0.0):
        check(lib.fvna_set_clock(self.handle, float(t), float(dt_next)))

    def fvna_step(self, nsteps):
        check(lib.fvna_step(self.handle, int(nsteps)))

    def fvna_sync(self, allow_device_errors=False):
        allow = (E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES) if allow_device_errors else ()
        return check(lib.fvna_sync(self.handle), allow)

    def fvna_shift(self, ncols):
        check(lib.fvna_shift(self.handle, int(ncols)))

    def fvna_step_window(self, window, state, nsteps):
        """window: fvna_window (t1 [s], check_every, quantum); state:
        fvna_window_state, updated in place."""
        check(lib.fvna_step_window(self.handle, ctypes.byref(window), ctypes.byref(state), int(nsteps)))

    def fvna_set_recorder(self, row=None, probe_col=-1, path_len=0, row_max=None, probe_t=None,
                          probe_rho=None):
        """row None stops recording; otherwise row_max (path_len doubles) and the
        probe arrays are device tensors (torch, float64) that must outlive the
        recording."""
        if row is None:
            check(lib.fvna_set_recorder(self.handle, None))
            self._rec_keep = None
            return
        cap = 0 if probe_t is None else int(probe_t.numel())
        r = fvna_recorder(int(row), int(probe_col), int(path_len), row_max.data_ptr(),
                          probe_t.data_ptr() if probe_t is not None else None,
                          probe_rho.data_ptr() if probe_rho is not None else None, cap)
        self._rec_keep = (row_max, probe_t, probe_rho)
        check(lib.fvna_set_recorder(self.handle, ctypes.byref(r)))

    def fvna_get_state(self, allow_device_errors=False):
        out = [np.empty(self.shape, dtype=np.float64) for _ in range(3)]
        allow = (E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES) if allow_device_errors else ()
        check(lib.fvna_get_state(self.handle, *[_dptr(a) for a in out]), allow)
        return tuple(out)

    def fvna_get_window(self, i0, j0, ni, nj, allow_device_errors=False):
        out = [np.empty((int(nj), int(ni)), dtype=np.float64) for _ in range(3)]
        allow = (E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES) if allow_device_errors else ()
        check(lib.fvna_get_window(self.handle, int(i0), int(j0), int(ni), int(nj),
                                  *[_dptr(a) for a in out]), allow)
        return tuple(out)

    def fvna_get_stats(self, allow_device_errors=False):
        s = fvna_stats()
        allow = (E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES) if allow_device_errors else ()
        check(lib.fvna_get_stats(self.handle, ctypes.byref(s)), allow)
        return {k: getattr(s, k) for k, _ in fvna_stats._fields_}

    def fvna_sums(self):
        out = np.zeros(3)
        check(lib.fvna_sums(self.handle, _dptr(out)))
        return out

    def fvna_taylor_errors(self, front0_x_m, front0_y_m, half_length_m):
        """(E1, Einf) of eq. (error) on the line along the Taylor profile's
        propagation direction centred on its analytic front (device, FP64)."""
        out = np.zeros(2)
        check(lib.fvna_taylor_errors(self.handle, float(front0_x_m), float(front0_y_m), float(half_length_m),
                                     _dptr(out)))
        return float(out[0]), float(out[1])

    def fvna_time_step_kernel(self, reps):
        ms = ctypes.c_double()
        check(lib.fvna_time_step_kernel(self.handle, int(reps), ctypes.byref(ms)))
        return ms.value

    def fvna_autotune(self):
        tr = ctypes.c_int32()
        check(lib.fvna_autotune(self.handle, ctypes.byref(tr)))
        return tr.value

    def fvna_get_tile_rows(self):
        tr = ctypes.c_int32()
        check(lib.fvna_get_tile_rows(self.handle, ctypes.byref(tr)))
        return tr.value

    def fvna_destroy(self):
        if getattr(self, "handle", None):
            lib.fvna_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.fvna_destroy()
        except Exception:
            pass


class Batch:
    """Many independent simulations advanced by one batched launch per step."""

    def __init__(self, params_list, device="cuda:0", stream=None):
        import torch
        self.params = list(params_list)
        self.device = torch.device(device)
        n = len(self.params)
        arr = (fvna_params * n)(*self.params)
        self.bufs = []
        ptrs = (ctypes.c_void_p * (3 * n))()
        with torch.cuda.device(self.device):
            for k, p in enumerate(self.params):
                sb, xb = workspace_size(p)
                a = _device_buffer(sb, self.device)
                b = _device_buffer(sb, self.device)
                x = _device_buffer(xb, self.device)
                self.bufs += [a, b, x]
                ptrs[3 * k], ptrs[3 * k + 1], ptrs[3 * k + 2] = a.data_ptr(), b.data_ptr(), x.data_ptr()
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(lib.fvna_batch_create(n, arr, ptrs, _stream_handle(self.stream), ctypes.byref(h)))
        self.handle = h
        self.n = n

    def fvna_batch_set_state(self, k, rho_p, mom_x, mom_y):
        p = self.params[k]
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (rho_p, mom_x, mom_y)]
        for a in arrs:
            if a.shape != (p.ny, p.nx):
                raise ValueError("state shape mismatch")
        check(lib.fvna_batch_set_state(self.handle, int(k), *[_dptr(a) for a in arrs]))

    def fvna_batch_step(self, nsteps):
        check(lib.fvna_batch_step(self.handle, int(nsteps)))

    def fvna_batch_sync(self):
        return check(lib.fvna_batch_sync(self.handle))

    def fvna_batch_get_state(self, k):
        p = self.params[k]
        out = [np.empty((p.ny, p.nx), dtype=np.float64) for _ in range(3)]
        check(lib.fvna_batch_get_state(self.handle, int(k), *[_dptr(a) for a in out]))
        return tuple(out)

    def fvna_batch_get_stats(self, k):
        s = fvna_stats()
        check(lib.fvna_batch_get_stats(self.handle, int(k), ctypes.byref(s)))
        return {k2: getattr(s, k2) for k2, _ in fvna_stats._fields_}

    def fvna_batch_time_step_kernel(self, reps):
        ms = ctypes.c_double()
        check(lib.fvna_batch_time_step_kernel(self.handle, int(reps), ctypes.byref(ms)))
        return ms.value

    def fvna_batch_autotune(self):
        out = (ctypes.c_int32 * self.n)()
        check(lib.fvna_batch_autotune(self.handle, out))
        return list(out)

    def fvna_batch_get_tile_rows(self):
        out = (ctypes.c_int32 * self.n)()
        check(lib.fvna_batch_get_tile_rows(self.handle, out))
        return list(out)

    def fvna_batch_destroy(self):
        if getattr(self, "handle", None):
            lib.fvna_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.fvna_batch_destroy()
        except Exception:
            pass


def make_source(freq, p_surface, focal_length, aperture, ramp_cycles=3.0, envelope="ramp",
                packet_cycles=4.0, stage2_time=None):
    env = ENVELOPES[envelope] if isinstance(envelope, str) else int(envelope)
    return fvna_source(float(freq), float(p_surface), float(focal_length), float(aperture),
                       float(ramp_cycles), env, float(packet_cycles), int(stage2_time is not None),
                       float(stage2_time) if stage2_time is not None else 0.0)


def fvna_sums_noalloc(params, state, out, stream=None):
    """FP64 sums of one state buffer (a device tensor laid out as the library
    stores a state) into `out` (a device float64 tensor of 3 elements), on
    `stream` (default: torch's current stream); asynchronous."""
    check(lib.fvna_sums_noalloc(ctypes.byref(params), ctypes.c_void_p(state.data_ptr()),
                                _stream_handle(stream), ctypes.c_void_p(out.data_ptr())))


def sim_from_workload(w, device="cuda:0", precision=None, **over):
    """Create a Sim for a workload dict of paper_1311_3004_amd.inputs and load its state."""
    kw = dict(bc=w["bc"], geometry=w["geometry"], precision=precision or w["precision"],
              cfl_target=w.get("cfl_target", 0.9), cfl_max=w.get("cfl_max", 1.0))
    kw.update(over)
    p = make_params(w["nx"], w["ny"], w["dx"], w["medium"], **kw)
    s = Sim(p, device=device)
    if "source" in w:
        src = w["source"]
        s.fvna_set_source(0, src["freq"], src["p_surface"], src["focal_length"], src["aperture"],
                          src.get("ramp_cycles", 3.0), src.get("envelope", "ramp"),
                          src.get("packet_cycles", 4.0), src.get("stage2_time"))
    if "taylor" in w:
        t = w["taylor"]
        s.fvna_set_taylor(t["amplitude_pa"], t.get("x0_m", 0.0), t.get("angle", 0.0))
    s.fvna_set_state(*w["state"])
    if w.get("t0", 0.0) != 0.0:
        # keep a first step given in the parameters (fvna_set_clock recomputes
        # it from the state when dt_next <= 0)
        s.fvna_set_clock(w["t0"], p.dt0 if p.dt0 > 0 else 0.0)
    return s
