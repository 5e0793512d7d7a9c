"""Full-size workloads on the GPU, in the launch configuration bench.py times.

* gaussian-pulse 4096^2: FP64 and FP32 against the oracle on the full grid
  for two steps (every output element compared), FP32 against FP64 after
  2000 steps (max |dp|/p_peak).
* batch of uneven simulations: one batched launch per step is bitwise equal
  to separate contexts; the autotuner changes speed, never results.
* hifu-axisym 8192x2048 (20000 steps): FP32, FP16- and BF16-storage against
  the FP64 GPU path -- focal peak p+/p-, harmonics 1..5 at the focal cell over
  the final 5 cycles, shock-front position.  Tolerances are the measured
  errors with a margin; the FP64 path itself is held to the oracle by
  test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest

from common import max_rel, run_oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gaussian():
    from paper_1311_3004_amd import inputs
    return inputs.c2_pulse_fp32(4096, 4096)


DT_FULL = 0.9 * 1e-4 / 1500.0 / 1.001


@pytest.fixture(scope="module")
def gaussian_oracle(orc, gaussian):
    _say("case: oracle, gaussian 4096^2, 2 steps (CPU)")
    o, info = run_oracle(orc, gaussian, 2, fixed_dt=True, dt_si=DT_FULL)
    assert info["status"] == 0
    return o


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_gaussian_4096_two_steps_vs_oracle(gaussian, gaussian_oracle, precision, tol):
    from paper_1311_3004_amd import fvna
    w = gaussian
    med = w["medium"]
    _say(f"case: gaussian 4096^2 {precision} 2 steps vs oracle (fixed dt)")
    s = fvna.sim_from_workload(w, precision=precision, fixed_dt=True, dt0=DT_FULL)
    s.fvna_step(2)
    rp, mx, my = s.fvna_get_state()
    g = (rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"]))
    err = max_rel(g, gaussian_oracle)
    _say(f"  max rel err {err:.3e}")
    assert err <= tol
    s.fvna_destroy()


def test_gaussian_4096_fp32_vs_fp64_2000_steps(gaussian):
    from paper_1311_3004_amd import fvna
    w = gaussian
    out = {}
    for prec in ("f64", "f32"):
        _say(f"case: gaussian 4096^2 {prec} 2000 adaptive steps")
        s = fvna.sim_from_workload(w, precision=prec)
        s.fvna_step(2000)
        out[prec] = (s.fvna_get_state()[0], s.fvna_get_stats())
        s.fvna_destroy()
    a, sa = out["f64"]
    b, sb = out["f32"]
    err = float(np.max(np.abs(a - b)) / np.max(np.abs(a)))
    _say(f"  fp32 max |dp|/p_peak {err:.3e}")
    assert sa["steps"] == sb["steps"] == 2000
    assert abs(sa["t"] - sb["t"]) <= 1e-8 * sa["t"]
    assert err <= 1e-5          # the FP32 accuracy target on this workload


def _batch_sims():
    from paper_1311_3004_amd import inputs
    rng = np.random.default_rng(44)
    sims = []
    for k, (nx, ny) in enumerate([(300, 260), (517, 129), (64, 400), (1000, 96), (133, 133), (257, 511)]):
        med = dict(inputs.WATER, beta=float(rng.uniform(3, 5)), delta=float(10 ** rng.uniform(-6, -5)))
        med, rp, mx, my, c = inputs.gaussian_pulse(nx, ny, 1e-4, float(rng.uniform(0.1e6, 5e6)), 20.0, 0.0,
                                                   medium=med, rng=rng)
        sims.append({"nx": nx, "ny": ny, "dx": 1e-4, "medium": med, "state": (rp, mx, my),
                     "bc": ("extrap0", "reflect", "periodic", "periodic") if k % 2 else ("extrap0",) * 4})
    return sims


@pytest.mark.parametrize("precision,geometry", [("f32", "planar"), ("f64", "planar"), ("f32", "axisym"),
                                                ("f64", "axisym")])
def test_batched_equals_separate_contexts_bitwise(precision, geometry):
    """Each member of a batch equals the same simulation run alone, bit for
    bit; the axisymmetric batch also checks every member's own per-row 1/r
    table (the rows of the members differ)."""
    from paper_1311_3004_amd import fvna
    sims = _batch_sims()
    if geometry == "axisym":
        for x in sims:
            x["bc"] = ("extrap0", "extrap0", "reflect", "extrap0")
    plist = [fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], geometry=geometry,
                              precision=precision, tile_rows=[16, 40, 96][k % 3]) for k, x in enumerate(sims)]
    _say(f"case: batch of {len(sims)} {precision} {geometry}")
    B = fvna.Batch(plist)
    for k, x in enumerate(sims):
        B.fvna_batch_set_state(k, *x["state"])
    B.fvna_batch_step(60)
    B.fvna_batch_sync()
    for k, x in enumerate(sims):
        s = fvna.Sim(fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], geometry=geometry,
                                      precision=precision))
        s.fvna_set_state(*x["state"])
        s.fvna_step(60)
        a = s.fvna_get_state()
        b = B.fvna_batch_get_state(k)
        sa, sb = s.fvna_get_stats(), B.fvna_batch_get_stats(k)
        assert sa["steps"] == sb["steps"] == 60 and sa["t"] == sb["t"]
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
        s.fvna_destroy()
    B.fvna_batch_destroy()


def test_batch_autotune_changes_speed_not_results():
    """fvna_batch_autotune picks heights per size class by timing the batch;
    the batch then still equals separate contexts bit for bit, and a new batch
    of the same composition starts with the chosen heights."""
    from paper_1311_3004_amd import fvna
    sims = _batch_sims()
    plist = [fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], precision="f32")
             for x in sims]
    _say(f"case: batch autotune, {len(sims)} members")
    B = fvna.Batch(plist)
    for k, x in enumerate(sims):
        B.fvna_batch_set_state(k, *x["state"])
    tr = B.fvna_batch_autotune()
    assert tr == B.fvna_batch_get_tile_rows() and all(t in (32, 48, 64, 96, 128, 192, 256) for t in tr)
    B.fvna_batch_step(40)
    B.fvna_batch_sync()
    for k, x in enumerate(sims):
        s = fvna.Sim(plist[k])
        s.fvna_set_state(*x["state"])
        s.fvna_step(40)
        for u, v in zip(s.fvna_get_state(), B.fvna_batch_get_state(k)):
            assert np.array_equal(u, v)
        s.fvna_destroy()
    B.fvna_batch_destroy()
    B2 = fvna.Batch(plist)
    assert B2.fvna_batch_get_tile_rows() == tr
    B2.fvna_batch_destroy()


def test_autotune_changes_speed_not_results():
    from paper_1311_3004_amd import fvna, inputs
    w = inputs.c2_pulse_fp32(1024, 768)
    _say("case: autotune")
    a = fvna.sim_from_workload(w, precision="f32", tile_rows=24)
    a.fvna_step(40)
    ra = a.fvna_get_state()
    b = fvna.sim_from_workload(w, precision="f32")
    tr = b.fvna_autotune()
    assert tr == b.fvna_get_tile_rows() and tr >= 16
    b.fvna_step(40)
    rb = b.fvna_get_state()
    for u, v in zip(ra, rb):
        assert np.array_equal(u, v)


@pytest.fixture(scope="module")
def hifu_runs():
    """The hifu-axisym 8192x2048 workload (0.2 MPa) in every precision."""
    from paper_1311_3004_amd import fvna, inputs, diagnostics as dg
    w = inputs.c3_hifu_fp32()
    med, src = w["medium"], w["source"]
    a = src["p_surface"] / (med["rho0"] * med["c0"] ** 2)
    res = {}
    for prec in ("f64", "f32", "f32_f16store", "f32_bf16store"):
        _say(f"case: hifu-axisym 8192x2048 {prec} 20000 steps")
        over = {"store_scale": (64 * a,) * 3} if "store" in prec else {}
        s = fvna.sim_from_workload(w, precision=prec, **over)
        t, P = dg.record_row(s, w["steps"], 5.0 / src["freq"])
        st = s.fvna_get_stats()
        row = s.fvna_get_window(0, 0, w["nx"], 1)[0][0] * med["c0"] ** 2
        s.fvna_destroy()
        assert st["status"] == 0 and st["steps"] == w["steps"]
        res[prec] = (t, P, row, st)
    return w, res


def _focal(w, res, prec, zstar=None):
    from paper_1311_3004_amd import diagnostics as dg
    t, P, row, st = res[prec]
    f = dg.focal_summary(t, P, w["source"]["freq"], w["dx"], zstar=zstar)
    f["front"] = dg.shock_front(row, f["z_index"], 300)
    return f


# The error budget of each storage precision on this workload against the
# FP64 run (focal p+ and p- relative, harmonics 1-5 relative, phase lag of the
# shock front in cells, by least-squares alignment of the axial profiles,
# diagnostics.front_shift); None: the precision does not resolve that quantity
# and no bound is claimed.  FP16 storage resolves the focal pressures, the
# first three harmonics and the front; BF16 (8-bit significand) only the focal
# pressures, to about 2% -- its harmonics are off by 12-280% and its front by
# 2-8 cells.  Half-width storage rounds every cell of every step, so these
# errors move with rounding-level changes: of the FP32 arithmetic (two builds
# that differ only there: BF16 p+ 2.7e-3 and 7.8e-3, p- 1.1e-3 and 9.3e-3) and
# of the storage scale (56 a ... 72 a: FP16 p+/- <= 3.0e-3, harmonics 1-3 <=
# 1.4e-3 / 5.4e-3 / 2.0e-2, lag <= 0.08 cells; BF16 p+/- 1.1e-3 ... 1.8e-2);
# the bounds hold for all of them.
@pytest.mark.parametrize("prec,tol_peak,tol_h,tol_front", [
    ("f32", 1e-4, [1e-4, 1e-3, 1e-3, 1e-3, 5e-3], 0.05),
    ("f32_f16store", 5e-3, [5e-3, 1e-2, 3e-2, None, None], 0.5),
    ("f32_bf16store", 2.5e-2, [None] * 5, None),
])
def test_hifu_axisym_precisions_against_fp64(hifu_runs, prec, tol_peak, tol_h, tol_front):
    from paper_1311_3004_amd import diagnostics as dg
    w, res = hifu_runs
    ref = _focal(w, res, "f64")
    # the focused field: pre-focal peak with gain well above 10 and p+ > |p-|
    assert ref["p_plus"] > 10 * w["source"]["p_surface"] and ref["p_plus"] > abs(ref["p_minus"])
    got = _focal(w, res, prec, zstar=ref["z_index"])
    c = dg.compare(got, ref)
    lag = dg.front_shift(res[prec][2], res["f64"][2], int(round(ref["front"])))
    _say(f"  {prec}: p+ {c['p_plus_rel']:.2e} p- {c['p_minus_rel']:.2e} "
         f"harmonics {['%.1e' % h for h in c['harmonics_rel']]} front lag {lag} cells "
         f"(steepest gradient {got['front'] - ref['front']:+.3f})")
    assert c["p_plus_rel"] <= tol_peak and c["p_minus_rel"] <= tol_peak
    for h, tol in zip(c["harmonics_rel"], tol_h):
        if tol is not None:
            assert h <= tol
    if tol_front is not None:
        assert lag is not None and abs(lag) <= tol_front


ETAS = (20, 40, 80)


@pytest.fixture(scope="module")
def packet_runs():
    """The focused wave packet of Sec. 4.2 (aperture a = 10, F = 50, 60
    wavelengths long) at 20, 40 and 80 cells per wavelength (the paper uses
    20, 41, 82), FP64: on-axis pressure maxima and the probe at (1, 0)."""
    from paper_1311_3004_amd import fvna, inputs, diagnostics as dg
    res = {}
    for eta in ETAS:
        w = inputs.hifu_packet(eta=eta, a=10.0, length_wl=60.0, margin_wl=10.0)
        _say(f"case: {w['name']} FP64 to t_end")
        s = fvna.sim_from_workload(w, precision="f64")
        pmax, t, p = dg.axis_maxima(s, w["t_end"], probe_col=eta - 1)
        st = s.fvna_get_stats()
        s.fvna_destroy()
        assert st["status"] == 0
        res[eta] = {"x": (np.arange(w["nx"]) + 0.5) / eta, "pmax": pmax, "t": t, "p": p, "stats": st,
                    "w": w}
    return res


def test_packet_axis_maxima_converge_second_order(packet_runs):
    """The paper finds second-order convergence of the on-axis maxima
    against its reference (Table 2); without that reference, successive
    refinements must shrink at second order: log2(|p20 - p40| / |p40 - p80|)
    between 1.5 and 3 over the axis (2 to 58 wavelengths)."""
    e0, e1, e2 = ETAS
    xc = packet_runs[e0]["x"]
    sel = (xc > 2.0) & (xc < 58.0)
    pa = packet_runs[e0]["pmax"]
    pb = np.interp(xc, packet_runs[e1]["x"], packet_runs[e1]["pmax"])
    pc = np.interp(xc, packet_runs[e2]["x"], packet_runs[e2]["pmax"])
    d1 = np.mean(np.abs(pa - pb)[sel])
    d2 = np.mean(np.abs(pb - pc)[sel])
    order = np.log2(d1 / d2)
    _say(f"  axis maxima: |p{e0}-p{e1}| {d1:.4g} Pa, |p{e1}-p{e2}| {d2:.4g} Pa, order {order:.2f}; "
         f"relative to the peak {d2 / np.max(pc):.2e}")
    assert 1.5 < order < 3.0


def test_packet_focuses_and_keeps_the_cfl_band(packet_runs):
    """At 80 cells per wavelength the on-axis maximum lies before the
    geometric focus F = 50 (the focal shift of a finite aperture) with a gain
    over the source amplitude, and the CFL number stays within the paper's
    printed band for this experiment, std(nu) < 2.5e-4."""
    r = packet_runs[ETAS[-1]]
    x, pmax = r["x"], r["pmax"]
    p_s = r["w"]["source"]["p_surface"]
    k = int(np.argmax(pmax))
    _say(f"  eta {ETAS[-1]}: on-axis peak {pmax[k]/1e6:.3f} MPa at x1 = {x[k]:.2f} wavelengths "
         f"(gain {pmax[k]/p_s:.2f}); nu std {r['stats']['nu_std']:.2e}")
    assert 20.0 < x[k] < 50.0
    assert pmax[k] > 1.5 * p_s
    for eta in ETAS:
        assert packet_runs[eta]["stats"]["nu_std"] < 2.5e-4


def test_moving_domain_reproduces_the_fixed_domain_maxima():
    """The moving domain of Sec. 4 (24 wavelengths long, still until the
    packet centre reaches its middle at t1 = 12 periods, then following it in
    quarter-wavelength jumps; the source side extrapolating from t1 on) must
    give the on-axis maxima and the probe series at (1, 0) of a fixed
    60-wavelength domain with the same second stage, at 40 cells per
    wavelength, wherever neither run's edges can reach: the maxima before
    x1 = 52 (waves reflected by the fixed domain's right side at 60 meet the
    packet beyond 54) and the probe until t1 (from then on the moving domain's
    trailing edge approaches it).  There both agree to 1e-9 of their peaks,
    while the moving run updates 2.5 times fewer cells."""
    from paper_1311_3004_amd import fvna, inputs, diagnostics as dg
    eta = 40
    out = {}
    for win in (None, 24.0):
        w = inputs.hifu_packet(eta=eta, a=10.0, length_wl=60.0, margin_wl=10.0, window_wl=win)
        w["source"]["stage2_time"] = 12.0 / inputs.PACKET_FREQ
        _say(f"case: {w['name']} FP64 to t_end, second stage at 12 periods")
        s = fvna.sim_from_workload(w, precision="f64")
        out[win] = dg.axis_maxima(s, w["t_end"], probe_col=eta - 1, window=w.get("window"),
                                  path_cells=w["path_cells"]) + (s.fvna_get_stats(), w)
        s.fvna_destroy()
    pf, tf, prf, stf, _ = out[None]
    pw, tw, prw, stw, ww = out[24.0]
    assert stf["status"] == 0 and stw["status"] == 0 and stw["steps"] == stf["steps"]
    assert pw.shape == pf.shape and np.isfinite(pw).all()
    assert np.array_equal(tw, tf[: len(tw)]) and len(tw) > 0.2 * len(tf)
    x = (np.arange(ww["path_cells"]) + 0.5) / eta
    d = np.abs(pw - pf) / np.max(pf)
    k = int(np.argmax(d))
    err = np.max(d[x < 52.0])
    early = tw < ww["window"]["t1"]
    perr = np.max(np.abs(prw - prf[: len(prw)])[early]) / np.max(np.abs(prf))
    _say(f"  moving domain {ww['nx']}x{ww['ny']}: on-axis maxima rel err {err:.2e} before x1 = 52 "
         f"(largest {d[k]:.2e} at x1 = {x[k]:.1f}), probe {perr:.2e} before t1")
    assert err <= 1e-9 and perr <= 1e-9


def _table1():
    import math
    import os
    ang = {"0": 0.0, "pi/32": math.pi / 32, "pi/16": math.pi / 16, "pi/8": math.pi / 8, "pi/4": math.pi / 4}
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_taylor_shock.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        th, norm, *v = line.split()
        rows[(ang[th], norm)] = [float(x) for x in v]
    return rows


def test_taylor_shock_table1_theta0_row():
    """Sec. 4.1 on the GPU through the C ABI, FP64: the Taylor shock along
    x1 (analytic data on all four sides, a = 1e-7, eta cells per 10-90% rise
    of the profile, 100 of those units of travel, errors on the 10-unit line
    centred on the front) for eta = 5 ... 82 and nu_W = 0.6 ... 0.99.  The
    statistics of Table 1's theta_T = 0 row must come out as printed: rates
    to 0.05, the worst R^2 to 0.01, the eta = 82 errors to 10%; and std(nu)
    stays below the paper's 1e-8."""
    from paper_1311_3004_amd import taylor_report as tr
    rows = []
    for eta in tr.ETAS:
        for nu in tr.NUS:
            r = tr.run(0.0, eta, nu, "rise", "f64")
            assert r["status"] == 0 and r["t_over_t_end"] >= 1.0
            assert r["nu_std"] < 1e-8
            rows.append(r)
    _say(f"case: taylor shock theta_T = 0, {len(rows)} runs")
    want = _table1()
    for srow in tr.summarize(rows):
        ref = want[(0.0, srow["norm"])]
        got = [srow["rate_best"], srow["rate_worst"], srow["rate_mean"], srow["r2_worst"],
               srow["err_finest_best"], srow["err_finest_worst"]]
        _say(f"  {srow['norm']}: " + " ".join(f"{g:.4g}/{w:.4g}" for g, w in zip(got, ref)))
        for g, w in zip(got[:3], ref[:3]):
            assert abs(g - w) <= 0.05
        assert abs(got[3] - ref[3]) <= 0.01
        for g, w in zip(got[4:], ref[4:]):
            assert abs(g / w - 1.0) <= 0.10


@pytest.mark.parametrize("window_wl", [None, 16.0])
def test_recorder_matches_sampling_every_step(window_wl):
    """The device recorder (fvna_set_recorder) against copying the on-axis
    row out after every step, on the focused packet (20 cells per wavelength,
    a = 10, a 30-wavelength path) on a fixed and on a moving domain: the same
    steps, the same maxima bit for bit (on the moving domain the host copy
    also sees the zeros that enter, which can only raise a column's maximum
    from below zero to zero) and the same probe series."""
    import time
    from paper_1311_3004_amd import fvna, inputs, diagnostics as dg
    w = inputs.hifu_packet(eta=20, a=10.0, length_wl=30.0, margin_wl=5.0, window_wl=window_wl)
    out = []
    for fn in (dg.axis_maxima, dg.axis_maxima_recorded):
        _say(f"case: {w['name']} {fn.__name__}")
        s = fvna.sim_from_workload(w, precision="f64")
        t0 = time.time()
        res = fn(s, w["t_end"], probe_col=19, window=w.get("window"), path_cells=w["path_cells"])
        st = s.fvna_get_stats()
        out.append(res + (st, time.time() - t0))
        s.fvna_destroy()
    (ph, th, prh, sth, wh), (pd, td, prd, std_, wd) = out
    _say(f"  steps {sth['steps']} / {std_['steps']}, wall {wh:.2f} s / {wd:.2f} s")
    assert sth["steps"] == std_["steps"] and sth["t"] == std_["t"]
    assert np.all((ph == pd) | ((ph == 0.0) & (pd < 0.0)))
    assert np.max(pd) > 1e5
    n = min(len(th), len(td))
    assert abs(len(th) - len(td)) <= (0 if window_wl is None else 1) and n > 100
    assert np.array_equal(th[:n], td[:n]) and np.array_equal(prh[:n], prd[:n])


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 2e-6)])
def test_batched_members_vs_oracle(precision, tol):
    """The batch of 64 uneven simulations in the benchmark's launch
    configuration (library default tile height), 3 adaptive steps; the
    smallest, a middle and the largest member against the oracle run on that
    member alone (each with its own medium and time step)."""
    import oracle as orc
    from paper_1311_3004_amd import fvna, inputs
    sims = inputs.c4_batch()
    plist = [fvna.make_params(x["nx"], x["ny"], x["dx"], x["medium"], bc=x["bc"], precision=precision)
             for x in sims]
    _say(f"case: batch of {len(sims)} {precision}, 3 steps, members vs oracle")
    B = fvna.Batch(plist)
    for k, x in enumerate(sims):
        B.fvna_batch_set_state(k, *x["state"])
    B.fvna_batch_step(3)
    B.fvna_batch_sync()
    order = sorted(range(len(sims)), key=lambda k: sims[k]["nx"] * sims[k]["ny"])
    for k in (order[0], order[len(order) // 2], order[-1]):
        x = sims[k]
        med = x["medium"]
        rp, mx, my = B.fvna_batch_get_state(k)
        g = (rp / med["rho0"], mx / (med["rho0"] * med["c0"]), my / (med["rho0"] * med["c0"]))
        o, info = run_oracle(orc, x, 3)
        assert info["status"] == 0 and B.fvna_batch_get_stats(k)["steps"] == 3
        err = max_rel(g, o)
        _say(f"  member {k} {x['nx']}x{x['ny']}: max rel err {err:.3e}")
        assert err <= tol
    B.fvna_batch_destroy()
