"""Writes tests/golden/table1_mobile_oracle.txt: rows of the Taylor-shock
study of Sec. 4.1 (Table 1) on the mobile domain of Sec. 4, computed by the
FP64 oracle only (oracle.run_window, oracle.taylor_line_errors) from the
seeded input generators (inputs.taylor_oblique, inputs.taylor_oblique_window):
theta_T in {pi/8, pi/4}, eta in {5, 10, 20}, nu_W = 0.9, 100 units of travel,
the run stopped at the first state with t >= t_end.

    python tests/golden/make_table1_mobile.py      # a few minutes on 8 threads
"""
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1311_3004_amd import inputs  # noqa: E402

WINDOW_L = 24.0
CASES = [(th, eta, 0.9) for th in (math.pi / 8, math.pi / 4) for eta in (5, 10, 20)]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table1_mobile_oracle.txt")


def one(theta, eta, nu):
    w = inputs.taylor_oblique(eta, theta, cfl_target=nu)
    ww, win = inputs.taylor_oblique_window(w, WINDOW_L)
    med = ww["medium"]
    dx, c0 = ww["dx"], med["c0"]
    p = oracle.make_params_si(ww["nx"], ww["ny"], dx, c0, med["rho0"], med["beta"], med["delta"],
                              bc=("taylor",) * 4, cfl_target=nu, taylor_si=ww["taylor"])
    rp, mx, my = ww["state"]
    rc = med["rho0"] * c0
    state = (rp / med["rho0"], mx / rc, my / rc)
    t_end = ww["t_end"] * c0 / dx
    t1 = win["t1"] * c0 / dx
    t, dt, x_off, steps = 0.0, 0.0, 0, 0
    ce, q, sp = win["check_every"], win["quantum"], win["speed"]
    while t < t_end:
        R, M, N, info, xo = oracle.run_window(p, *state, ce, t, dt, t1, ce, q, x_off=x_off, speed=sp)
        assert info["status"] == 0
        if info["t"] < t_end:
            state, t, dt, x_off, steps = (R, M, N), info["t"], info["dt_next"], xo, steps + ce
            continue
        # the first state with t >= t_end lies inside this chunk: redo it one
        # step at a time (no check before the chunk ends, as in the chunk)
        s1, t_, dt_ = state, t, dt
        for k in range(1, ce + 1):
            if k == ce:
                s1, t_, dt_, x_off = (R, M, N), info["t"], info["dt_next"], xo
                break
            R1, M1, N1, i1, _ = oracle.run_window(p, *s1, 1, t_, dt_, t1, ce, q, x_off=x_off, speed=sp)
            assert i1["status"] == 0
            s1, t_, dt_ = (R1, M1, N1), i1["t"], i1["dt_next"]
            if t_ >= t_end:
                break
        state, t, steps = s1, t_, steps + k
    front0 = (ww["front0_m"][0] / dx, ww["front0_m"][1] / dx)
    e1, einf = oracle.taylor_line_errors(p, t, state[0], front0, 5.0 * ww["unit_m"] / dx, x_off=x_off)
    return steps, x_off, e1, einf


def main():
    oracle.set_threads(int(os.environ.get("ORACLE_THREADS", "8")))
    lines = ["# Taylor shock (Sec. 4.1, Table 1) on the mobile domain of Sec. 4, FP64 oracle:",
             "# window 24 units wide, Taylor data on all four sides anchored on the path, moving at",
             "# the front point's speed c0 cos(theta_T) in quarter-unit jumps after t1; errors of",
             "# eq. (error) on the 10-unit line along the propagation direction.",
             "# Written by tests/golden/make_table1_mobile.py (oracle only).",
             "# theta_T  eta  nu_W  steps  x_off  E1  Einf"]
    for theta, eta, nu in CASES:
        steps, xo, e1, einf = one(theta, eta, nu)
        e1, einf = float(e1), float(einf)
        lines.append(f"{theta!r} {eta} {nu!r} {steps} {xo} {e1!r} {einf!r}")
        print(lines[-1], flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
