"""Time-to-solution and on-axis results of the focused wave-packet experiment
(Sec. 4.2) at the paper's parameters.

For each (a, eta, nu_W) the packet is run from t = -6 periods to t = 100 (it
travels 100 wavelengths) over a path 105 wavelengths long and a domain a + 10
wide -- either a fixed domain over the whole path or (window) the moving
domain of Sec. 4, 24 wavelengths long -- sampling the cells next to the
symmetry line every step (on the device, fvna_set_recorder).  One JSON line per
run: wall time (including the sampling), steps, cell-updates per second,
the on-axis peak pressure and its position, the CFL statistics and the
amplitudes of harmonics 1..8 at the probe (x1, x2) = (1, 0).

    python -m paper_1311_3004_amd.packet_report                 # the paper's extremes
    python -m paper_1311_3004_amd.packet_report all             # a x eta x nu_W of Sec. 4.2
    python -m paper_1311_3004_amd.packet_report all f32
    python -m paper_1311_3004_amd.packet_report all f64 window
    python -m paper_1311_3004_amd.packet_report 30,82,0.99 f32 window    # one case
"""
import itertools
import json
import sys
import time

import numpy as np

from . import diagnostics as dg
from . import fvna, inputs

A_VALUES = (10.0, 20.0, 30.0)
ETAS = (20, 41, 82)
NUS = (0.6, 0.7, 0.8, 0.9, 0.99)
EXTREMES = ((30.0, 20, 0.99), (30.0, 82, 0.99), (30.0, 82, 0.6))


WINDOW_WL = 24.0


def run(a, eta, nu, precision="f64", t_end_periods=100.0, length_wl=105.0, window_wl=None):
    w = inputs.hifu_packet(eta=eta, a=a, length_wl=length_wl, margin_wl=10.0, cfl_target=nu,
                           precision=precision, window_wl=window_wl)
    w["t_end"] = t_end_periods / inputs.PACKET_FREQ
    t0 = time.time()
    s = fvna.sim_from_workload(w, precision=precision)
    pmax, t, p = dg.axis_maxima_recorded(s, w["t_end"], probe_col=eta - 1, window=w.get("window"),
                                         path_cells=w["path_cells"])
    st = s.fvna_get_stats()
    s.fvna_destroy()
    elapsed = time.time() - t0
    x = (np.arange(w["path_cells"]) + 0.5) / eta
    k = int(np.argmax(pmax))
    return {"a": a, "eta": eta, "nu_W": nu, "precision": precision, "nx": w["nx"], "ny": w["ny"],
            "window_wl": window_wl,
            "status": st["status"], "steps": st["steps"], "wall_s": elapsed,
            "gcell_s": w["nx"] * w["ny"] * st["steps"] / elapsed / 1e9,
            "nu_mean": st["nu_mean"], "nu_std": st["nu_std"],
            "axis_peak_pa": float(pmax[k]), "axis_peak_x_wl": float(x[k]),
            "harmonics_at_1_0_pa": [float(h) for h in dg.spectrum(t, p, inputs.PACKET_FREQ, 8)]}


def main(argv):
    which = argv[1] if len(argv) > 1 else "extremes"
    precision = argv[2] if len(argv) > 2 else "f64"
    window_wl = WINDOW_WL if len(argv) > 3 and argv[3] == "window" else None
    if which == "extremes":
        cases = EXTREMES
    elif which == "all":
        cases = list(itertools.product(A_VALUES, ETAS, NUS))
    else:
        a, eta, nu = which.split(",")
        cases = [(float(a), int(eta), float(nu))]
    for a, eta, nu in cases:
        print(json.dumps(run(a, eta, nu, precision, window_wl=window_wl)), flush=True)


if __name__ == "__main__":
    main(sys.argv)
