"""Plain FP64 CPU oracle for the finite-volume step of Velasco-Segura & Rendon
(arXiv:1311.3004) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The product library never calls it and shares no
code with it.  The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA
contraction); this module only marshals arguments and converts SI units to the
dimensionless variables of the paper's renormalisation (Sec. 3, eqs. renorm and
phi-tdelta) with the reference length taken as the mesh spacing.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVALID, E_NOMEM, E_NONHYPERBOLIC, E_NONFINITE, E_RETRIES = 0, 1, 2, 4, 5, 6
BC = {"periodic": 0, "extrap0": 1, "reflect": 2, "taylor": 3, "source": 4}
GEOM = {"planar": 0, "axisym": 1}


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("beta", ctypes.c_double), ("delta", ctypes.c_double),
        ("geometry", ctypes.c_int), ("bc", ctypes.c_int * 4),
        ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double),
        ("max_retries", ctypes.c_int), ("fixed_dt", ctypes.c_int),
        ("taylor_amp", ctypes.c_double), ("taylor_width", ctypes.c_double),
        ("taylor_x0", ctypes.c_double), ("taylor_y0", ctypes.c_double),
        ("taylor_angle", ctypes.c_double),
        ("src_amp", ctypes.c_double), ("src_freq", ctypes.c_double),
        ("src_focal", ctypes.c_double), ("src_aperture", ctypes.c_double),
        ("src_ramp_cycles", ctypes.c_double),
        ("src_envelope", ctypes.c_int), ("src_packet_cycles", ctypes.c_double),
        ("src_stage2_on", ctypes.c_int), ("src_stage2", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("dt_next", ctypes.c_double), ("nu_last", ctypes.c_double),
        ("nu_mean", ctypes.c_double), ("nu_std", ctypes.c_double),
        ("steps", ctypes.c_long), ("rejected", ctypes.c_long),
        ("status", ctypes.c_int), ("status_step", ctypes.c_long),
    ]


def build(force=False):
    """Compile oracle.c into liboracle.so with gcc (FP64, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_roe.restype = ctypes.c_int
        L.orc_roe.argtypes = [d, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_mc.restype = d
        L.orc_mc.argtypes = [d]
        L.orc_flux.restype = None
        L.orc_flux.argtypes = [d, dp, dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.POINTER(Params), dp, dp, dp, ctypes.c_long, dp, dp,
                              ctypes.POINTER(Stats), dp]
        L.orc_dry_smax.restype = d
        L.orc_dry_smax.argtypes = [ctypes.POINTER(Params), dp, dp, dp, d]
        L.orc_taylor_value.restype = None
        L.orc_taylor_value.argtypes = [ctypes.POINTER(Params), d, d, d, dp]
        L.orc_source_g.restype = d
        L.orc_source_g.argtypes = [ctypes.POINTER(Params), d, d]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_get_threads.restype = ctypes.c_int
        L.orc_get_threads.argtypes = []
        L.orc_ghost.restype = ctypes.c_int
        L.orc_ghost.argtypes = [ctypes.POINTER(Params), dp, dp, dp, d, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, dp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def roe(beta, qL, qR):
    """Roe decomposition at one x1-interface (Sec. 3.2).  Returns a dict with
    s (3,), r (3 waves x 3 comps), alpha (3,), W (3x3), amdq, apdq, or None
    when the speeds are not real."""
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    s = np.zeros(3); r = np.zeros((3, 3)); al = np.zeros(3); W = np.zeros((3, 3))
    am = np.zeros(3); ap = np.zeros(3)
    ok = lib().orc_roe(float(beta), _ptr(qL), _ptr(qR), _ptr(s), _ptr(r), _ptr(al), _ptr(W),
                       _ptr(am), _ptr(ap))
    if not ok:
        return None
    return {"s": s, "r": r, "alpha": al, "W": W, "amdq": am, "apdq": ap}


def mc(theta):
    return lib().orc_mc(float(theta))


def flux(beta, q):
    """x1 flux of eq. adim:q with the constant ambient pressure removed."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.zeros(3)
    lib().orc_flux(float(beta), _ptr(q), _ptr(f))
    return f


def make_params(nx, ny, beta, delta, bc=("extrap0",) * 4, geometry="planar",
                cfl_target=0.9, cfl_max=1.0, max_retries=8, fixed_dt=False,
                taylor=None, source=None):
    """Dimensionless parameters.  delta is delta~ = delta/(c0 dx).  taylor: dict
    amp, width, x0, y0, angle (cells).  source: dict amp, freq (cycles per
    dx/c0), focal, aperture (cells), ramp_cycles, envelope ("ramp" or
    "packet"), packet_cycles, stage2 (time from which the whole side x- is
    zero-order extrapolation; None: never)."""
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.beta, p.delta = float(beta), float(delta)
    p.geometry = GEOM[geometry] if isinstance(geometry, str) else int(geometry)
    for k, b in enumerate(bc):
        p.bc[k] = BC[b] if isinstance(b, str) else int(b)
    p.cfl_target, p.cfl_max = float(cfl_target), float(cfl_max)
    p.max_retries, p.fixed_dt = int(max_retries), int(bool(fixed_dt))
    t = taylor or {}
    p.taylor_amp = float(t.get("amp", 0.0)); p.taylor_width = float(t.get("width", 1.0))
    p.taylor_x0 = float(t.get("x0", 0.0)); p.taylor_y0 = float(t.get("y0", 0.0))
    p.taylor_angle = float(t.get("angle", 0.0))
    s = source or {}
    p.src_amp = float(s.get("amp", 0.0)); p.src_freq = float(s.get("freq", 1.0))
    p.src_focal = float(s.get("focal", 1e30)); p.src_aperture = float(s.get("aperture", 0.0))
    p.src_ramp_cycles = float(s.get("ramp_cycles", 3.0))
    p.src_envelope = {"ramp": 0, "packet": 1}[s.get("envelope", "ramp")]
    p.src_packet_cycles = float(s.get("packet_cycles", 4.0))
    st2 = s.get("stage2")
    p.src_stage2_on = int(st2 is not None)
    p.src_stage2 = float(st2) if st2 is not None else 0.0
    return p


def make_params_si(nx, ny, dx, c0, rho0, beta, delta, bc=("extrap0",) * 4, geometry="planar",
                   cfl_target=0.9, cfl_max=1.0, max_retries=8, fixed_dt=False,
                   taylor_si=None, source_si=None):
    """SI parameters -> dimensionless ones (length unit dx, time unit dx/c0,
    density unit rho0, velocity unit c0, pressure unit rho0 c0^2)."""
    p0 = rho0 * c0 * c0
    taylor = None
    if taylor_si is not None:
        a = taylor_si["amplitude_pa"] / p0
        # width of the tanh profile: delta~_L / beta = a with L = width (eq. OurTaylorS)
        width = (delta / c0) / (beta * a) / dx
        taylor = {"amp": a, "width": width, "x0": taylor_si.get("x0_m", 0.0) / dx,
                  "y0": taylor_si.get("y0_m", 0.0) / dx, "angle": taylor_si.get("angle", 0.0)}
    source = None
    if source_si is not None:
        source = {"amp": source_si["p_surface"] / p0, "freq": source_si["freq"] * dx / c0,
                  "focal": source_si["focal_length"] / dx, "aperture": source_si["aperture"] / dx,
                  "ramp_cycles": source_si.get("ramp_cycles", 3.0),
                  "envelope": source_si.get("envelope", "ramp"),
                  "packet_cycles": source_si.get("packet_cycles", 4.0),
                  "stage2": (None if source_si.get("stage2_time") is None
                             else source_si["stage2_time"] * c0 / dx)}
    return make_params(nx, ny, beta, delta / (c0 * dx), bc, geometry, cfl_target, cfl_max,
                       max_retries, fixed_dt, taylor, source)


def run(p, R, M, N, nsteps, t=0.0, dt=0.0, want_hist=False):
    """Advance (R, M, N) (arrays [ny][nx], dimensionless) by nsteps accepted
    steps.  Returns (R, M, N, info) with info holding status, t, dt_next,
    nu statistics and (optionally) the nu history."""
    R = np.array(R, dtype=np.float64, order="C", copy=True)
    M = np.array(M, dtype=np.float64, order="C", copy=True)
    N = np.array(N, dtype=np.float64, order="C", copy=True)
    assert R.shape == (p.ny, p.nx) and M.shape == R.shape and N.shape == R.shape
    tt = ctypes.c_double(t)
    dd = ctypes.c_double(dt)
    st = Stats()
    hist = np.zeros(max(int(nsteps), 1))
    e = lib().orc_run(ctypes.byref(p), _ptr(R), _ptr(M), _ptr(N), int(nsteps), ctypes.byref(tt),
                      ctypes.byref(dd), ctypes.byref(st), _ptr(hist) if want_hist else None)
    info = {"status": e, "t": st.t, "dt_next": st.dt_next, "nu_last": st.nu_last,
            "nu_mean": st.nu_mean, "nu_std": st.nu_std, "steps": st.steps,
            "rejected": st.rejected, "status_step": st.status_step}
    if want_hist:
        info["nu_hist"] = hist[: st.steps].copy()
    return R, M, N, info


def dry_smax(p, R, M, N, t=0.0):
    R = np.ascontiguousarray(R, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    return lib().orc_dry_smax(ctypes.byref(p), _ptr(R), _ptr(M), _ptr(N), float(t))


def taylor_value(p, x, y, t):
    q = np.zeros(3)
    lib().orc_taylor_value(ctypes.byref(p), float(x), float(y), float(t), _ptr(q))
    return q


def source_g(p, r, t):
    return lib().orc_source_g(ctypes.byref(p), float(r), float(t))


def set_threads(n):
    """Worker threads of the oracle's sweeps and source (OpenMP over rows; the
    result is bitwise the same for every count).  Default 1."""
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


def ghost(p, R, M, N, t, side, gi, gj, layer):
    """(R, M, N) of ghost cell (gi, gj), layer `layer` of side `side` (0: x-, 1: x+,
    2: y-, 3: y+) at time t, by that side's boundary rule from the interior state."""
    R = np.ascontiguousarray(R, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    assert R.shape == (p.ny, p.nx) and M.shape == R.shape and N.shape == R.shape
    q = np.zeros(3)
    e = lib().orc_ghost(ctypes.byref(p), _ptr(R), _ptr(M), _ptr(N), float(t), int(side), int(gi),
                        int(gj), int(layer), _ptr(q))
    if e != OK:
        raise ValueError(f"orc_ghost: error {e} for side {side}, cell ({gi}, {gj}), layer {layer}")
    return q


__all__ = ["build", "lib", "roe", "mc", "flux", "make_params", "make_params_si", "run",
           "dry_smax", "taylor_value", "source_g", "ghost", "set_threads", "get_threads", "BC", "GEOM", "Params", "Stats"]


def shift(R, M, N, ncols, fill=None):
    """Move the domain ncols cells along +x1 (the moving domain of Sec. 4):
    column i of the result is column i + ncols of the input; the ncols columns
    that enter on the right hold undisturbed medium: R = M = N = 0, or, with
    fill given, the three columns fill(i) returns for new column i."""
    out = []
    for F in (R, M, N):
        G = np.zeros_like(F)
        if ncols < F.shape[1]:
            G[:, : F.shape[1] - ncols] = F[:, ncols:]
        out.append(G)
    if fill is not None:
        nx = R.shape[1]
        for i in range(max(nx - ncols, 0), nx):
            col = fill(i)
            for G, c in zip(out, col):
                G[:, i] = c
    return out[0], out[1], out[2]


def _window_params(p, x_off, x0_path):
    """Parameters of the domain after it moved x_off cells: the Taylor profile
    is anchored on the path, so in domain coordinates its x0 moves back by
    x_off (column i of the domain is path column x_off + i)."""
    q = Params.from_buffer_copy(p)
    q.taylor_x0 = x0_path - x_off
    return q


def run_window(p, R, M, N, nsteps, t, dt, t1, check_every, quantum, x_off=0, speed=1.0):
    """The two stages of Sec. 4 on a moving domain.  Steps are taken in
    chunks of check_every accepted steps; after each chunk, once t >= t1 (the
    wave has reached the middle of the domain), the domain origin is moved to
    quantum * floor((t - t1) speed / quantum) cells (the domain follows the
    wave at `speed` cells per unit time -- 1 for c0 -- in jumps of quantum
    cells).  Analytic (Taylor) data stay on the path: every side uses the
    profile at path coordinates, and with a Taylor side x+ the entering
    columns hold the profile at the time of the move.  p's taylor_x0 is the
    path coordinate of the profile (domain origin at path column x_off on
    entry).  Returns (R, M, N, info, x_off)."""
    done = 0
    info = None
    x0_path = p.taylor_x0
    taylor_right = p.bc[1] == BC["taylor"]
    while done < nsteps:
        k = min(check_every, nsteps - done)
        q = _window_params(p, x_off, x0_path)
        R, M, N, info = run(q, R, M, N, k, t=t, dt=dt)
        if info["status"] != OK:
            return R, M, N, info, x_off
        t, dt = info["t"], info["dt_next"]
        done += k
        if k == check_every and t >= t1:
            target = quantum * int(np.floor((t - t1) * speed / quantum))
            if target > x_off:
                fill = None
                if taylor_right:
                    qn = _window_params(p, target, x0_path)
                    ys = np.arange(p.ny) + 0.5

                    def fill(i, qn=qn, tt=t):
                        v = np.array([taylor_value(qn, i + 0.5, y, tt) for y in ys])
                        return v[:, 0], v[:, 1], v[:, 2]
                R, M, N = shift(R, M, N, target - x_off, fill)
                x_off = target
    return R, M, N, info, x_off


def taylor_line_errors(p, t, R, front0, half_length, x_off=0):
    """E1 and Einf of eq. (error) (Sec. 4.1) of the dimensionless density
    perturbation R ([ny][nx] of a domain that has moved x_off cells) against
    the Taylor profile of p (taylor_value, p's taylor_x0 on the path) at time
    t: over the cells of the straight line of length 2 half_length along the
    propagation direction, centred on the analytic front front0 + t (cos, sin)
    (reading R9: one cell per column, the cell the line crosses there; one per
    row when the line is steeper than 45 degrees), E1 = sum |R - R_ref| /
    sum |R_ref|, Einf = max |R - R_ref| / max |R_ref|.  Lengths in cells, time
    in dx/c0.  Plain loops, test infrastructure only."""
    import math
    c, s = math.cos(p.taylor_angle), math.sin(p.taylor_angle)
    fx, fy = front0[0] + t * c, front0[1] + t * s
    ny, nx = R.shape
    cells = []
    if abs(c) >= abs(s):
        for i in range(math.ceil(fx - half_length * c - 0.5), math.floor(fx + half_length * c - 0.5) + 1):
            cells.append((i, math.floor(fy + (i + 0.5 - fx) * s / c)))
    else:
        for j in range(math.ceil(fy - half_length * s - 0.5), math.floor(fy + half_length * s - 0.5) + 1):
            cells.append((math.floor(fx + (j + 0.5 - fy) * c / s), j))
    num = den = big = bigref = 0.0
    for i, j in cells:
        if not (0 <= i - x_off < nx and 0 <= j < ny):
            continue
        ref = taylor_value(p, i + 0.5, j + 0.5, t)[0]
        e = abs(R[j, i - x_off] - ref)
        num += e
        den += abs(ref)
        big = max(big, e)
        bigref = max(bigref, abs(ref))
    return num / den, big / bigref
