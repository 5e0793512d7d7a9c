"""The Taylor-shock study of Sec. 4.1 (Table 1) on the GPU: for every
propagation angle theta_T, mesh parameter eta and nu_W the shock travels 100
units (FP64 by default), and the errors E1, Einf of eq. (error) are read on
the 10-unit line along the propagation direction centred on the analytic
front.  Convergence rates are the slopes of the linear regressions of
log E against log eta over eta = 5 ... 82, with their R^2.

    python -m paper_1311_3004_amd.taylor_report              # all 125 runs, reading "rise"
    python -m paper_1311_3004_amd.taylor_report all tanh      # the other reading of the unit
    python -m paper_1311_3004_amd.taylor_report 0.3927,41,0.9 rise f32   # one run
    python -m paper_1311_3004_amd.taylor_report all rise f64 window      # on the mobile domain

The mobile domain of Sec. 4 (last argument "window"): WINDOW_L units wide
with the fixed run's height, Taylor data on all four sides in both stages
(anchored on the path), still until the front point -- the point of the
front on the error line's axis -- reaches the middle column, then moving
along x1 at that point's speed c0 cos(theta_T) in quarter-unit jumps, so
that the error line stays centred in the window.  The errors are computed
on the device (fvna_taylor_errors) in path coordinates.

One JSON line per run, then one summary line per (theta_T, norm) with the
statistics Table 1 prints: best / worst / mean rate over nu_W, worst R^2,
best / worst error at eta = 82.
"""
import itertools
import json
import math
import sys
import time

import numpy as np

from . import diagnostics as dg
from . import fvna, inputs

THETAS = (0.0, math.pi / 32, math.pi / 16, math.pi / 8, math.pi / 4)
ETAS = (5, 10, 20, 41, 82)
NUS = (0.6, 0.7, 0.8, 0.9, 0.99)


WINDOW_L = 24.0           # width of the mobile domain in units L


def run(theta, eta, nu, reading="rise", precision="f64", mobile=False):
    w = inputs.taylor_oblique(eta, theta, cfl_target=nu, reading=reading, precision=precision)
    window = None
    if mobile:
        w, window = inputs.taylor_oblique_window(w, WINDOW_L)
    t_wall = time.time()
    s = fvna.sim_from_workload(w, precision=precision)
    t_end = w["t_end"]
    if window is not None:
        win = fvna.fvna_window(window["t1"], window["check_every"], window["quantum"], window["speed"])
        ws = fvna.fvna_window_state(0, 0)
    while True:
        st = s.fvna_get_stats()
        if st["t"] >= t_end or st["status"] != 0:
            break
        left = (t_end - st["t"]) / st["dt_next"]
        n = max(1, int(left) - 2) if left > 4 else 1
        if window is None:
            s.fvna_step(n)
        else:
            s.fvna_step_window(win, ws, n)
    st = s.fvna_get_stats()
    e1, einf = s.fvna_taylor_errors(w["front0_m"][0], w["front0_m"][1], 5.0 * w["unit_m"])
    s.fvna_destroy()
    wall = time.time() - t_wall
    out = {"theta": theta, "eta": eta, "nu_W": nu, "reading": reading, "precision": precision,
           "domain": "mobile" if mobile else "fixed",
           "nx": w["nx"], "ny": w["ny"], "status": st["status"], "steps": st["steps"],
           "rejected": st["rejected"], "t_over_t_end": st["t"] / t_end, "nu_mean": st["nu_mean"],
           "nu_std": st["nu_std"], "E1": e1, "Einf": einf, "wall_s": wall,
           "gcell_s": w["nx"] * w["ny"] * st["steps"] / wall / 1e9}
    if window is not None:
        out["x_off"] = int(ws.x_off)
    return out


def summarize(rows):
    """Table 1's statistics per theta and norm."""
    out = []
    for theta in sorted({r["theta"] for r in rows}):
        for norm in ("E1", "Einf"):
            rates, r2s, e82 = [], [], []
            for nu in sorted({r["nu_W"] for r in rows}):
                pts = sorted((r["eta"], r[norm]) for r in rows if r["theta"] == theta and r["nu_W"] == nu)
                if len(pts) < 2:
                    continue
                x = np.log([p[0] for p in pts])
                y = np.log([p[1] for p in pts])
                slope, icpt = np.polyfit(x, y, 1)
                res = y - (slope * x + icpt)
                r2 = 1.0 - np.sum(res ** 2) / np.sum((y - y.mean()) ** 2)
                rates.append(-slope)
                r2s.append(r2)
                e82 += [p[1] for p in pts if p[0] == max(q[0] for q in pts)]
            if rates:
                out.append({"theta": theta, "norm": norm, "rate_best": max(rates), "rate_worst": min(rates),
                            "rate_mean": float(np.mean(rates)), "r2_worst": min(r2s),
                            "err_finest_best": min(e82), "err_finest_worst": max(e82),
                            "finest_eta": max(r["eta"] for r in rows)})
    return out


def main(argv):
    which = argv[1] if len(argv) > 1 else "all"
    reading = argv[2] if len(argv) > 2 else "rise"
    precision = argv[3] if len(argv) > 3 else "f64"
    mobile = len(argv) > 4 and argv[4] == "window"
    if which == "all":
        cases = list(itertools.product(THETAS, ETAS, NUS))
    else:
        th, eta, nu = which.split(",")
        cases = [(float(th), int(eta), float(nu))]
    rows = []
    for theta, eta, nu in cases:
        r = run(theta, eta, nu, reading, precision, mobile)
        rows.append(r)
        print(json.dumps(r), flush=True)
    for srow in summarize(rows):
        print(json.dumps({"summary": srow}), flush=True)


if __name__ == "__main__":
    main(sys.argv)
