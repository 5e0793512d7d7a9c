"""Shared helpers of the test-suite: run one workload on the oracle and on the
HIP library with the same seeded inputs."""
import numpy as np


def dimless_state(w):
    med = w["medium"]
    rp, mx, my = w["state"]
    return rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"])


def oracle_params(orc, w, fixed_dt=False, **over):
    med = w["medium"]
    kw = dict(bc=w["bc"], geometry=w["geometry"], cfl_target=w.get("cfl_target", 0.9),
              cfl_max=w.get("cfl_max", 1.0), fixed_dt=fixed_dt,
              taylor_si=w.get("taylor"), source_si=w.get("source"))
    kw.update(over)
    return orc.make_params_si(w["nx"], w["ny"], w["dx"], med["c0"], med["rho0"], med["beta"],
                              med["delta"], **kw)


def run_oracle(orc, w, steps, fixed_dt=False, dt_si=0.0, **over):
    """Returns (R, M, N) dimensionless and the info dict."""
    med = w["medium"]
    p = oracle_params(orc, w, fixed_dt=fixed_dt, **over)
    R, M, N = dimless_state(w)
    dt = dt_si * med["c0"] / w["dx"] if dt_si > 0 else 0.0
    t0 = w.get("t0", 0.0) * med["c0"] / w["dx"]
    R1, M1, N1, info = orc.run(p, R, M, N, steps, t=t0, dt=dt, want_hist=True)
    return (R1, M1, N1), info


def run_gpu(w, steps, precision="f64", fixed_dt=False, dt_si=0.0, tile_rows=0, sim=None, **over):
    """Returns (R, M, N) dimensionless, the stats dict and the Sim."""
    from paper_1311_3004_amd import fvna
    med = w["medium"]
    if sim is None:
        sim = fvna.sim_from_workload(w, precision=precision, fixed_dt=fixed_dt, dt0=dt_si,
                                     tile_rows=tile_rows, **over)
    sim.fvna_step(steps)
    rp, mx, my = sim.fvna_get_state()
    st = sim.fvna_get_stats()
    return (rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"])), st, sim


def max_rel(a, b, peak=None):
    """max |a - b| over the three fields, relative to the peak |R| of b."""
    peak = peak if peak is not None else max(np.max(np.abs(b[0])), 1e-300)
    return max(float(np.max(np.abs(x - y))) for x, y in zip(a, b)) / peak


def pulse_workload(nx, ny, bc, geometry="planar", seed=7, amplitude_pa=2e6, noise=0.005,
                   sigma_cells=8.0, dx=1e-4, medium=None, source=None, taylor=None):
    """Small Gaussian-pulse workload with the given boundaries (for parity cases)."""
    from paper_1311_3004_amd import inputs
    med, rp, mx, my, c = inputs.gaussian_pulse(nx, ny, dx, amplitude_pa, sigma_cells, noise, seed,
                                               medium=medium)
    rng = np.random.default_rng(seed + 1000)
    # give the pulse some momentum so every component is exercised
    mx = mx + 0.3 * rp * med["c0"] * rng.uniform(-1, 1)
    my = my + 0.2 * rp * med["c0"] * rng.uniform(-1, 1)
    w = {"name": "pulse", "nx": nx, "ny": ny, "dx": dx, "medium": med, "bc": tuple(bc),
         "geometry": geometry, "precision": "f64", "cfl_target": 0.9, "cfl_max": 1.0,
         "state": (rp, mx, my)}
    if source is not None:
        w["source"] = source
    if taylor is not None:
        w["taylor"] = taylor
    return w
