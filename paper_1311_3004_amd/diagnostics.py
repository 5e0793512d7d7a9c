"""Diagnostics of a running simulation: on-axis probes, focal peak, harmonics
and shock-front position (the quantities the paper reads off its focused-wave
runs: on-axis pressure maxima and the spectrum at a point, Sec. 4.2).

Everything here post-processes states the library hands out through
fvna_get_window; none of it is part of the time step.
"""
import math

import numpy as np


def record_row(sim, total_steps, tail_time, row=0, margin=1.15):
    """Advance `sim` to `total_steps` accepted steps (counted from its current
    state) and sample row `row` of p' = c0^2 rho' after every step of the final
    `tail_time` seconds.  Returns (t [n], p [n, nx]) with t the sample times."""
    p = sim.params
    c2 = p.c0 * p.c0
    st = sim.fvna_get_stats()
    dt = st["dt_next"]
    n_tail = min(total_steps, int(math.ceil(margin * tail_time / dt)) + 2)
    sim.fvna_step(total_steps - n_tail)
    ts, ps = [], []
    for _ in range(n_tail):
        sim.fvna_step(1)
        rp, _, _ = sim.fvna_get_window(0, row, p.nx, 1)
        ts.append(sim.fvna_get_stats()["t"])
        ps.append(rp[0] * c2)
    t = np.array(ts)
    P = np.array(ps)
    keep = t >= t[-1] - tail_time * (1 + 1e-9)
    return t[keep], P[keep]


def harmonics(t, p, freq, n=5):
    """Amplitudes of harmonics 1..n of p(t) over the sampled window by a
    nonuniform DFT (trapezoidal weights), assuming the window spans an integer
    number of periods of `freq`."""
    t = np.asarray(t)
    w = np.empty_like(t)
    w[1:-1] = 0.5 * (t[2:] - t[:-2])
    w[0] = 0.5 * (t[1] - t[0])
    w[-1] = 0.5 * (t[-1] - t[-2])
    T = t[-1] - t[0]
    out = []
    for k in range(1, n + 1):
        e = np.exp(-2j * np.pi * k * freq * t)
        out.append(abs(2.0 / T * np.sum(w * p * e)))
    return np.array(out)


def focal_summary(t, P, freq, dx, n_harm=5, zstar=None):
    """p+ and p- per axial cell over the window, the focal cell (largest p+)
    and the harmonics there."""
    pplus = P.max(axis=0)
    pminus = P.min(axis=0)
    k = int(np.argmax(pplus)) if zstar is None else int(zstar)
    return {"z_index": k, "z_m": (k + 0.5) * dx, "p_plus": float(pplus[k]), "p_minus": float(pminus[k]),
            "p_plus_axis": pplus, "p_minus_axis": pminus,
            "harmonics": harmonics(t, P[:, k], freq, n_harm)}


def shock_front(p_row, center, half_width):
    """Sub-cell position of the steepest compression front (largest -dp/dz)
    of an axial pressure profile within [center - half_width, center + half_width],
    refined by a parabola through the three largest-gradient samples."""
    g = -(p_row[1:] - p_row[:-1])                 # at faces k + 1/2 (cell units, k = 0..)
    lo = max(1, center - half_width)
    hi = min(len(g) - 1, center + half_width)
    k = lo + int(np.argmax(g[lo:hi]))
    y0, y1, y2 = g[k - 1], g[k], g[k + 1]
    den = y0 - 2 * y1 + y2
    off = 0.5 * (y0 - y2) / den if den != 0 else 0.0
    return k + 1.0 + off                         # face k + 1/2 sits at cell coordinate k + 1


def front_shift(p_row, ref_row, center, half_width=40, max_shift=8.0):
    """Phase lag of an axial pressure profile against a reference, in cells:
    the shift s minimising the sum over |z - center| <= half_width of
    (p_row[z] - ref(z - s))^2, ref linearly interpolated (s > 0: p_row is
    ahead).  Scanned in 0.01-cell steps over |s| <= max_shift and refined by
    a parabola through the three smallest sums.  It uses the whole front
    rather than three gradient samples (shock_front): on the 8192 x 2048
    focused-source run with FP16 storage, two builds that differ only in FP32
    rounding put the steepest-gradient position +0.28 and -0.63 cells from
    the FP64 run's, and this lag at -0.06 and -0.01.  None when the best shift
    lies on the edge of the scan."""
    p_row = np.asarray(p_row, dtype=np.float64)
    ref_row = np.asarray(ref_row, dtype=np.float64)
    c = int(center)
    pad = half_width + int(np.ceil(max_shift)) + 1
    if c - pad < 0 or c + pad >= min(len(p_row), len(ref_row)):
        raise ValueError("front_shift: window outside the profile")
    z = np.arange(c - half_width, c + half_width + 1, dtype=np.float64)
    n = int(round(max_shift / 0.01))
    S = np.arange(-n, n + 1) * 0.01
    R = np.interp((z[None, :] - S[:, None]).ravel(), np.arange(len(ref_row)), ref_row).reshape(len(S), len(z))
    E = np.sum((p_row[c - half_width:c + half_width + 1][None, :] - R) ** 2, axis=1)
    i = int(np.argmin(E))
    if i == 0 or i == len(S) - 1:
        return None
    e0, e1, e2 = E[i - 1], E[i], E[i + 1]
    den = e0 - 2 * e1 + e2
    return float(S[i] + (0.5 * 0.01 * (e0 - e2) / den if den > 0 else 0.0))


def compare(a, b):
    """Relative differences of focal quantities of run a against reference b."""
    h = np.abs(a["harmonics"] - b["harmonics"]) / np.maximum(b["harmonics"], 1e-300)
    return {"p_plus_rel": abs(a["p_plus"] - b["p_plus"]) / abs(b["p_plus"]),
            "p_minus_rel": abs(a["p_minus"] - b["p_minus"]) / abs(b["p_minus"]),
            "harmonics_rel": [float(x) for x in h]}


def axis_maxima(sim, t_end, probe_col=None, row=0, max_steps=10 ** 7, window=None, path_cells=None):
    """Advance `sim` one step at a time until its time reaches t_end and
    return the largest pressure p' = c0^2 rho' seen at each cell of row `row`
    (the cells next to the symmetry line: the on-axis pressure maxima of Sec.
    4.2), and the time series (t, p) at column probe_col of that row.

    window: a dict t1, check_every, quantum -- the domain moves (fvna_step_window)
    and the maxima are kept over path_cells columns of the path it covers
    (column x_off + i of the path is column i of the domain); the probe
    series stops when the domain has moved past probe_col."""
    p = sim.params
    c2 = p.c0 * p.c0
    ncols = p.nx if window is None else int(path_cells)
    pmax = np.full(ncols, -np.inf)
    ts, ps = [], []
    if window is not None:
        from . import fvna
        win = fvna.fvna_window(float(window["t1"]), int(window["check_every"]), int(window["quantum"]))
        state = fvna.fvna_window_state(0, 0)
    x_off = 0
    for _ in range(max_steps):
        st = sim.fvna_get_stats()
        if st["t"] >= t_end:
            break
        if window is None:
            sim.fvna_step(1)
        else:
            sim.fvna_step_window(win, state, 1)
            x_off = int(state.x_off)
        if x_off >= ncols:
            break
        rp, _, _ = sim.fvna_get_window(0, row, p.nx, 1)
        prow = rp[0] * c2
        n = min(p.nx, ncols - x_off)
        np.maximum(pmax[x_off:x_off + n], prow[:n], out=pmax[x_off:x_off + n])
        if probe_col is not None and x_off <= probe_col < x_off + p.nx:
            ts.append(sim.fvna_get_stats()["t"])
            ps.append(prow[probe_col - x_off])
    return pmax, np.array(ts), np.array(ps)


def spectrum(t, p, freq, n=8, packet_cycles=4.0):
    """Amplitudes of harmonics 1..n of a packet p(t) sampled at times t
    (nonuniform, the record covering the whole packet): the trapezoidal
    Fourier integral |2/D int p e^{-2 pi i k f t} dt| with D the equivalent
    duration of the envelope exp(-(f t / W)^10), int exp(-(f t / W)^10) dt =
    (2 W / f) Gamma(1.1), so that a carrier A w(t) sin(2 pi f t) gives A at
    k = 1 whatever the record length."""
    t = np.asarray(t)
    w = np.empty_like(t)
    w[1:-1] = 0.5 * (t[2:] - t[:-2])
    w[0] = 0.5 * (t[1] - t[0])
    w[-1] = 0.5 * (t[-1] - t[-2])
    D = 2.0 * packet_cycles * math.gamma(1.1) / freq
    return np.array([abs(2.0 / D * np.sum(w * p * np.exp(-2j * np.pi * k * freq * t)))
                     for k in range(1, n + 1)])

def line_cells(w, t, half_length=5.0, x_off=0, nx=None):
    """Cells on the line along the propagation direction of the oblique
    Taylor workload, half_length L on each side of the analytic front at time
    t: one cell per column (per row when the line is steeper than 45 degrees),
    the cell containing the line's point there.  Returns (i, j) path index
    arrays; on a domain that has moved x_off cells (nx columns wide) only the
    cells inside it are kept.  The direction cosines come from the C library's
    cos and sin, as the GPU library's (math.cos, not numpy's vector code)."""
    c, s = math.cos(w["theta"]), math.sin(w["theta"])
    dx, L = w["dx"], w["unit_m"]
    c0 = w["medium"]["c0"]
    fx = w["front0_m"][0] + c0 * t * c
    fy = w["front0_m"][1] + c0 * t * s
    if abs(c) >= abs(s):
        i = np.arange(int(np.ceil((fx - half_length * L * c) / dx - 0.5)),
                      int(np.floor((fx + half_length * L * c) / dx - 0.5)) + 1)
        y = fy + ((i + 0.5) * dx - fx) * s / c
        j = np.floor(y / dx).astype(int)
    else:
        j = np.arange(int(np.ceil((fy - half_length * L * s) / dx - 0.5)),
                      int(np.floor((fy + half_length * L * s) / dx - 0.5)) + 1)
        x = fx + ((j + 0.5) * dx - fy) * c / s
        i = np.floor(x / dx).astype(int)
    nx = w["nx"] if nx is None else nx
    keep = (i - x_off >= 0) & (i - x_off < nx) & (j >= 0) & (j < w["ny"])
    return i[keep], j[keep]


def taylor_errors(w, t, R, x_off=0):
    """E1 and Einf of eq. (error) for the oblique Taylor workload: the
    dimensionless perturbation R = rho'/rho0 on the cells of line_cells,
    against -a tanh((xi - c0 t)/w) at their centres, relative to the
    reference's own norms.  R is the [ny][nx] field of a domain that has
    moved x_off cells (0: fixed); the line is in path coordinates."""
    i, j = line_cells(w, t, x_off=x_off, nx=R.shape[1])
    c, s = math.cos(w["theta"]), math.sin(w["theta"])
    dx = w["dx"]
    xi = ((i + 0.5) * dx - w["taylor"]["x0_m"]) * c + (j + 0.5) * dx * s
    ref = -w["amplitude"] * np.tanh((xi - w["medium"]["c0"] * t) / w["tanh_unit_m"])
    num = R[j, i - x_off]
    d = np.abs(num - ref)
    return float(np.sum(d) / np.sum(np.abs(ref))), float(np.max(d) / np.max(np.abs(ref)))


def axis_maxima_recorded(sim, t_end, probe_col=None, row=0, window=None, path_cells=None, margin=1.05):
    """axis_maxima with the library's recorder (fvna_set_recorder): the
    maxima and the probe series are kept on the device after every step and
    read once at the end, so the steps run back to back (the stopping rule
    is the same: the first state with t >= t_end).  The maxima agree with
    axis_maxima wherever the wave has passed; at columns that entered a
    moving domain empty and saw only negative values since, axis_maxima also
    counts the 0 that entered."""
    import torch
    from . import fvna
    p = sim.params
    c2 = p.c0 * p.c0
    ncols = p.nx if window is None else int(path_cells)
    st = sim.fvna_get_stats()
    cap = 0
    if probe_col is not None:
        cap = int((t_end - st["t"]) / st["dt_next"] * margin) + 64
    dev = sim.device
    row_max = torch.full((ncols,), -math.inf, dtype=torch.float64, device=dev)
    probe_t = torch.full((cap,), math.nan, dtype=torch.float64, device=dev) if cap else None
    probe_rho = torch.full((cap,), math.nan, dtype=torch.float64, device=dev) if cap else None
    torch.cuda.synchronize(dev)
    sim.fvna_set_recorder(row, -1 if probe_col is None else probe_col, ncols, row_max, probe_t, probe_rho)
    if window is not None:
        win = fvna.fvna_window(float(window["t1"]), int(window["check_every"]), int(window["quantum"]))
        state = fvna.fvna_window_state(0, 0)
    try:
        while True:
            st = sim.fvna_get_stats()
            if st["t"] >= t_end:
                break
            left = (t_end - st["t"]) / st["dt_next"]
            n = max(1, int(left) - 2) if left > 4 else 1
            if window is None:
                sim.fvna_step(n)
            else:
                sim.fvna_step_window(win, state, n)
                if state.x_off >= ncols:
                    break
        sim.fvna_sync()
    finally:
        sim.fvna_set_recorder(None)
    pmax = row_max.cpu().numpy() * c2
    if not cap:
        return pmax, np.array([]), np.array([])
    t = probe_t.cpu().numpy()
    r = probe_rho.cpu().numpy()
    keep = ~np.isnan(t)
    return pmax, t[keep], r[keep] * c2
