"""Seeded synthetic workloads (initial conditions and SI parameters).

This module holds no arithmetic of the finite-volume method: it only draws
the seeded initial states and restates the five water-like workloads as plain
dictionaries.  It is shared by the tests (which feed the same arrays to the
HIP library and to the FP64 oracle) and by the benchmark.  Every random
number comes from numpy's PCG64 (``numpy.random.default_rng``).

Units are SI throughout: fields are (rho' [kg/m^3], rho*u [kg/m^2/s],
rho*v [kg/m^2/s]) on a row-major [ny][nx] grid with x1 contiguous; cell (i, j)
has its centre at ((i + 1/2) dx, (j + 1/2) dx).
"""
import numpy as np

WATER = {"c0": 1500.0, "rho0": 1000.0, "beta": 3.5, "delta": 4.3e-6}


def _medium(**over):
    m = dict(WATER)
    m.update(over)
    return m


def _p0(med):
    return med["rho0"] * med["c0"] ** 2


def taylor_step(nx=256, ny=256, dx=1e-4, amplitude_pa=1e6, x0_cells=64.0, noise=0.01,
                seed=1, medium=None):
    """Plane tanh pressure step of amplitude A (the jump is 2A) centred on a
    cell face, right-going (momentum equal to rho0 c0 times the unperturbed
    density ratio), with i.i.d. uniform multiplicative density noise
    R <- R (1 + noise * xi), xi ~ U[-1, 1).  Returns (medium, rho_p, mx, my)."""
    med = medium or _medium()
    a = amplitude_pa / _p0(med)
    width = (med["delta"] / med["c0"]) / (med["beta"] * a) / dx
    x = np.arange(nx) + 0.5
    R0 = -a * np.tanh((x - x0_cells) / width)
    R0 = np.broadcast_to(R0, (ny, nx)).copy()
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(ny, nx))
    R = R0 * (1.0 + noise * xi)
    rho_p = med["rho0"] * R
    mx = med["rho0"] * med["c0"] * R0
    my = np.zeros_like(R)
    return med, rho_p, mx, my


def gaussian_pulse(nx, ny, dx=1e-4, amplitude_pa=2e6, sigma_cells=20.0, noise=0.005, seed=2,
                   centre_box=None, medium=None, rng=None):
    """Gaussian density pulse R = a exp(-|x - xc|^2 / (2 sigma^2)) at rest, with
    the centre drawn on a cell centre inside centre_box = ((i0, i1), (j0, j1))
    (default: the middle half of the grid), plus additive white noise
    noise * a * xi, xi ~ U[-1, 1) per cell.  Returns (medium, rho_p, mx, my, centre)."""
    med = medium or _medium()
    a = amplitude_pa / _p0(med)
    rng = rng if rng is not None else np.random.default_rng(seed)
    if centre_box is None:
        centre_box = ((nx // 4, nx - nx // 4), (ny // 4, ny - ny // 4))
    ci = int(rng.integers(centre_box[0][0], centre_box[0][1]))
    cj = int(rng.integers(centre_box[1][0], centre_box[1][1]))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    d2 = (x[None, :] - (ci + 0.5)) ** 2 + (y[:, None] - (cj + 0.5)) ** 2
    R = a * np.exp(-d2 / (2.0 * sigma_cells ** 2))
    if noise:
        R = R + noise * a * rng.uniform(-1.0, 1.0, size=(ny, nx))
    rho_p = med["rho0"] * R
    return med, rho_p, np.zeros_like(R), np.zeros_like(R), (ci, cj)


# --------------------------------------------------------------------------
# The five workloads.  Each returns a dict with the SI parameters, the
# boundary kinds per side (x-, x+, y-, y+), the step count and the initial
# fields.  Grid sizes can be scaled down for tests with the keyword arguments.
# --------------------------------------------------------------------------

def c1_taylor_fp64(nx=256, ny=256, seed=1):
    """Plain method, FP64: 256x256, dx = 1e-4 m, tanh step of 1 MPa at x = 64 dx,
    1% noise, periodic in y, zero-order extrapolation in x, 200 adaptive steps."""
    med, rp, mx, my = taylor_step(nx, ny, 1e-4, 1e6, 64.0 * nx / 256.0, 0.01, seed)
    return {"name": "taylor-step 256x256 fp64", "nx": nx, "ny": ny, "dx": 1e-4, "medium": med,
            "bc": ("extrap0", "extrap0", "periodic", "periodic"), "geometry": "planar",
            "precision": "f64", "steps": 200, "cfl_target": 0.9, "cfl_max": 1.0,
            "state": (rp, mx, my)}


RISE_10_90 = 2.0 * np.arctanh(0.8)     # 10%-90% rise of tanh, in tanh units (2.197)


def taylor_oblique(eta, theta, cfl_target=0.9, reading="rise", amplitude=1e-7, travel=100.0,
                   margin=6.0, precision="f64", medium=None):
    """The Taylor-shock study of Sec. 4.1: p'/p0 = -a tanh((xi - c0 t)/w) with
    xi the distance along the propagation direction (cos theta, sin theta),
    a = 1e-7 (the paper's delta~/beta), w = delta / (c0 beta a) the tanh unit;
    M = R cos theta, N = R sin theta (eq. OurTaylorS rotated); analytic data
    on all four sides.

    The paper's length unit L and mesh parameter eta = cells per L: reading
    "rise" takes L as the 10%-90% rise of the profile (2.197 tanh units, the
    paper's own definition of L), reading "tanh" takes L = w (the unit in
    which its formula tanh(x - t) is written).  The front starts through the
    point (margin, margin) L from the lower-left corner and travels `travel`
    L; the domain covers the whole path with `margin` L to spare, so the
    front never meets the sides.  The errors are read on the 10-L line along
    the propagation direction centred on the analytic front at t_end
    (eq. error)."""
    med = dict(WATER if medium is None else medium)
    w_t = med["delta"] / (med["c0"] * med["beta"] * amplitude)       # tanh unit [m]
    L = w_t * (RISE_10_90 if reading == "rise" else 1.0)
    dx = L / eta
    c, s = float(np.cos(theta)), float(np.sin(theta))
    if abs(s) < 1e-15:
        s = 0.0
    nx = int(np.ceil((2 * margin + travel * c) * eta))
    ny = int(np.ceil((2 * margin + travel * s) * eta))
    px, py = margin * L, margin * L                                  # front at t = 0
    x0 = px + py * s / c                                             # xi = 0 through (px, py)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    xi = (x[None, :] - x0) * c + y[:, None] * s
    R = -amplitude * np.tanh(xi / w_t)
    p0 = _p0(med)
    rp = R * med["rho0"]
    mom = R * med["rho0"] * med["c0"]
    return {"name": f"taylor-oblique theta={theta:.4f} eta={eta} {reading} {nx}x{ny}", "nx": nx, "ny": ny,
            "dx": dx, "medium": med, "bc": ("taylor",) * 4, "geometry": "planar", "precision": precision,
            "cfl_target": cfl_target, "cfl_max": 1.0,
            "taylor": {"amplitude_pa": amplitude * p0, "x0_m": x0, "angle": theta},
            "t_end": travel * L / med["c0"], "front0_m": (px, py), "unit_m": L, "tanh_unit_m": w_t,
            "eta": eta, "theta": theta, "amplitude": amplitude,
            "state": (rp, mom * c, mom * s)}


def taylor_oblique_window(w, width_l=24.0):
    """The oblique Taylor workload `w` (taylor_oblique) cut to a mobile domain
    width_l units L wide (path columns 0 .. nx_w - 1 at the start, the fixed
    run's height) and its window rule: t1 [s] when the front point
    front0 + c0 t (cos, sin) reaches the middle column, domain speed
    cos(theta) in units of c0 (the front point's speed along x1, which keeps
    the error line centred), moves in quarter-unit jumps checked every 4
    steps.  Returns (workload, window)."""
    eta = w["eta"]
    nxw = int(np.ceil(width_l * eta))
    rp, mx, my = w["state"]
    ww = dict(w, nx=nxw, state=(rp[:, :nxw].copy(), mx[:, :nxw].copy(), my[:, :nxw].copy()))
    c = float(np.cos(w["theta"]))
    t1 = (0.5 * nxw * w["dx"] - w["front0_m"][0]) / (w["medium"]["c0"] * c)
    window = {"t1": t1, "check_every": 4, "quantum": max(1, int(round(eta / 4))), "speed": c}
    return ww, window


def c2_pulse_fp32(nx=4096, ny=4096, seed=2):
    """FP32 Cartesian 4096^2: 2 MPa Gaussian (sigma 20 cells) at a seed-chosen
    centre in [1536, 2560)^2 plus 0.5% white noise, absorbing (zero-order
    extrapolation) sides, 2000 steps."""
    box = ((nx * 3) // 8, (nx * 5) // 8), ((ny * 3) // 8, (ny * 5) // 8)
    med, rp, mx, my, c = gaussian_pulse(nx, ny, 1e-4, 2e6, 20.0, 0.005, seed, centre_box=box)
    return {"name": f"gaussian-pulse {nx}x{ny} fp32", "nx": nx, "ny": ny, "dx": 1e-4,
            "medium": med, "bc": ("extrap0",) * 4, "geometry": "planar", "precision": "f32",
            "steps": 2000, "cfl_target": 0.9, "cfl_max": 1.0, "state": (rp, mx, my),
            "centre": c}


def hifu_axisym(nz=8192, nr=2048, dx=2e-5, p_surface=2e5, steps=20000, precision="f32"):
    """Axisymmetric (x1 = z, x2 = r) focused field: 1 MHz sinusoid on the z = 0
    plane over r <= 35 mm with the paraxial focusing delay of a 62.6 mm focal
    length, 3-cycle ramp, symmetry axis at r = 0, quiescent start."""
    med = _medium()
    z = np.zeros((nr, nz))
    src = {"freq": 1e6, "p_surface": p_surface, "focal_length": 62.6e-3, "aperture": 35e-3,
           "ramp_cycles": 3.0}
    return {"name": f"hifu-axisym {nz}x{nr}", "nx": nz, "ny": nr, "dx": dx, "medium": med,
            "bc": ("source", "extrap0", "reflect", "extrap0"), "geometry": "axisym",
            "precision": precision, "steps": steps, "cfl_target": 0.9, "cfl_max": 1.0,
            "source": src, "state": (z, z.copy(), z.copy())}


def c3_hifu_fp32():
    return hifu_axisym(8192, 2048, 2e-5, 2e5, 20000, "f32")


def c5_hifu_mixed(precision="f32_f16store"):
    return hifu_axisym(16384, 8192, 1e-5, 1e6, 40000, precision)


# Soft tissue of the focused wave-packet experiment (Sec. 4.2): c0, rho0,
# beta and the sound diffusivity delta, with the 1.1 MHz driving frequency.
SOFT_TISSUE = {"c0": 1540.0, "rho0": 1000.0, "beta": 4.8, "delta": 6.4117e-4}
PACKET_FREQ = 1.1e6


def hifu_packet(eta=20, a=30.0, length_wl=60.0, margin_wl=10.0, cfl_target=0.9, precision="f64",
                window_wl=None):
    """The focused wave-packet experiment of Sec. 4.2 (lengths in wavelengths,
    eta cells per wavelength): planar geometry, x1 along the propagation axis,
    x2 transverse over a + margin_wl with the symmetry line x2 = 0 reflecting;
    on x1 = 0 the source of eq. hifuBC over 0 <= x2 <= a with focal length
    F = 50, amplitude A = 4.217e-4 (1.00 MPa) and the packet envelope
    (half-width 4 periods); zero-order extrapolation elsewhere.  The run
    starts at t0 = -6 periods, where the envelope is 9e-26; t_end = length_wl +
    6.5 periods, when the whole packet has passed x1 = length_wl.

    window_wl None: a fixed domain length_wl long; the second stage (the whole
    border x1 = 0 extrapolating) starts at t = +6 periods, when the packet has
    left the source.  window_wl = L: the moving domain of Sec. 4, L
    wavelengths long: still until the packet centre reaches its middle at
    t1 = L/2 periods (also the start of the second stage), then following the
    packet at c0, checked and moved in quarter-wavelength jumps; length_wl is
    then the length of the path covered (w["path_cells"])."""
    med = dict(SOFT_TISSUE)
    lam = med["c0"] / PACKET_FREQ
    dx = lam / eta
    path = int(round(length_wl * eta))
    nx = path if window_wl is None else int(round(window_wl * eta))
    ny = int(round((a + margin_wl) * eta))
    z = np.zeros((ny, nx))
    t2 = (6.0 if window_wl is None else 0.5 * window_wl) / PACKET_FREQ
    src = {"freq": PACKET_FREQ, "p_surface": 4.217e-4 * _p0(med), "focal_length": 50.0 * lam,
           "aperture": a * lam, "envelope": "packet", "packet_cycles": 4.0, "stage2_time": t2}
    t0 = -6.0 / PACKET_FREQ
    t_end = (length_wl + 6.5) / PACKET_FREQ
    name = f"hifu-packet eta={eta} a={a:g} {nx}x{ny}" + ("" if window_wl is None else f" moving over {path}")
    w = {"name": name, "nx": nx, "ny": ny, "dx": dx,
         "medium": med, "bc": ("source", "extrap0", "reflect", "extrap0"), "geometry": "planar",
         "precision": precision, "cfl_target": cfl_target, "cfl_max": 1.0, "source": src,
         "t0": t0, "t_end": t_end, "wavelength": lam, "eta": eta, "path_cells": path,
         "state": (z, z.copy(), z.copy())}
    if window_wl is not None:
        q = max(4, int(round(eta / 4)))
        w["window"] = {"t1": t2, "check_every": q, "quantum": q}
    return w


def c4_batch(n=64, seed=4, size_range=(256, 2048), steps=1000):
    """64 independent Cartesian simulations with seed-drawn uneven grids,
    amplitude U(0.1, 5) MPa, beta U(3, 5), delta log-uniform in [1e-6, 1e-5]
    m^2/s, Gaussian pulse (sigma 20 cells, no noise) in the middle half,
    dx = 1e-4 m, extrapolating sides, per-simulation adaptive dt."""
    children = np.random.SeedSequence(seed).spawn(n)
    sims = []
    for k, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        nx = int(rng.integers(size_range[0], size_range[1] + 1))
        ny = int(rng.integers(size_range[0], size_range[1] + 1))
        amp = float(rng.uniform(0.1e6, 5e6))
        beta = float(rng.uniform(3.0, 5.0))
        delta = float(10.0 ** rng.uniform(-6.0, -5.0))
        med = _medium(beta=beta, delta=delta)
        med, rp, mx, my, c = gaussian_pulse(nx, ny, 1e-4, amp, 20.0, 0.0, medium=med, rng=rng)
        sims.append({"name": f"batch-{k} {nx}x{ny}", "nx": nx, "ny": ny, "dx": 1e-4,
                     "medium": med, "bc": ("extrap0",) * 4, "geometry": "planar",
                     "precision": "f32", "steps": steps, "cfl_target": 0.9, "cfl_max": 1.0,
                     "state": (rp, mx, my)})
    return sims
