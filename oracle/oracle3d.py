"""Plain FP64 CPU oracle of the 3-D extension (three sweeps, four conserved
components) -- TEST INFRASTRUCTURE ONLY: imported by the test-suite, never by
the product library.  The arithmetic is in oracle3d.c; this module builds it
with gcc and marshals arguments (dimensionless units: cells, dx/c0)."""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle3d.c")
_LIB = os.path.join(_HERE, "liboracle3d.so")
BC = {"periodic": 0, "extrap0": 1, "reflect": 2}


class Params3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("beta", ctypes.c_double), ("delta", ctypes.c_double), ("bc", ctypes.c_int * 6),
                ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double),
                ("max_retries", ctypes.c_int), ("fixed_dt", ctypes.c_int)]


class Stats3(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_next", ctypes.c_double), ("nu_last", ctypes.c_double),
                ("nu_mean", ctypes.c_double), ("nu_std", ctypes.c_double),
                ("steps", ctypes.c_long), ("rejected", ctypes.c_long), ("status", ctypes.c_int)]


def build(force=False):
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", _LIB, _SRC, "-lm"], check=True)
    return _LIB


_L = None


def lib():
    global _L
    if _L is None:
        build()
        L = ctypes.CDLL(_LIB)
        d, dp = ctypes.c_double, ctypes.POINTER(ctypes.c_double)
        L.o3_run.restype = ctypes.c_int
        L.o3_run.argtypes = [ctypes.POINTER(Params3), dp, dp, dp, dp, ctypes.c_long, dp, dp,
                             ctypes.POINTER(Stats3)]
        L.o3_flux.restype = None
        L.o3_flux.argtypes = [d, dp, dp]
        L.o3_roe.restype = ctypes.c_int
        L.o3_roe.argtypes = [d, dp, dp, dp, dp, dp, dp, dp]
        _L = L
    return _L


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(nx, ny, nz, beta, delta, bc=("extrap0",) * 6, cfl_target=0.9, cfl_max=1.0,
                max_retries=8, fixed_dt=False):
    p = Params3()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.beta, p.delta = float(beta), float(delta)
    for k, b in enumerate(bc):
        p.bc[k] = BC[b]
    p.cfl_target, p.cfl_max = float(cfl_target), float(cfl_max)
    p.max_retries, p.fixed_dt = int(max_retries), int(bool(fixed_dt))
    return p


def run(p, Q, nsteps, t=0.0, dt=0.0):
    """Q: four arrays [nz][ny][nx] (R, M1, M2, M3).  Returns (Q', info)."""
    Q = [np.array(a, dtype=np.float64, order="C", copy=True) for a in Q]
    for a in Q:
        assert a.shape == (p.nz, p.ny, p.nx)
    tt, dd, st = ctypes.c_double(t), ctypes.c_double(dt), Stats3()
    e = lib().o3_run(ctypes.byref(p), *[_ptr(a) for a in Q], int(nsteps), ctypes.byref(tt),
                     ctypes.byref(dd), ctypes.byref(st))
    return Q, {"status": e, "t": st.t, "dt_next": st.dt_next, "steps": st.steps, "rejected": st.rejected,
               "nu_mean": st.nu_mean, "nu_std": st.nu_std}


def roe(beta, qL, qR):
    s, al, amdq, apdq = np.zeros(4), np.zeros(4), np.zeros(4), np.zeros(4)
    W = np.zeros((4, 4))
    qL, qR = np.array(qL, dtype=float), np.array(qR, dtype=float)
    ok = lib().o3_roe(float(beta), _ptr(qL), _ptr(qR), _ptr(s), _ptr(al), _ptr(W), _ptr(amdq), _ptr(apdq))
    return ok, s, al, W, amdq, apdq
