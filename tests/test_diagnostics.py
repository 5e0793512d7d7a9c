"""Host-side post-processing of recorded series (no GPU)."""
import numpy as np

from paper_1311_3004_amd import diagnostics as dg


def test_packet_spectrum_recovers_the_carrier_amplitudes():
    """A packet A1 w(t) sin(2 pi f t) + A3 w(t) sin(6 pi f t + 0.3) with the
    envelope w of eq. hifuBC:g (W = 4 periods), sampled unevenly: harmonic 1
    gives A1 and harmonic 3 gives A3 (to the small overlap of the envelope's
    spectrum at neighbouring harmonics), harmonic 2 is empty, whatever the
    length of the record around the packet."""
    f, W, A1, A3 = 1.1e6, 4.0, 2.5e5, 4e3
    rng = np.random.default_rng(3)
    for t0, t1 in ((-6.5, 6.5), (-7.0, 100.0)):
        t = np.sort(rng.uniform(t0, t1, 40000)) / f
        env = np.exp(-(f * t / W) ** 10)
        p = env * (A1 * np.sin(2 * np.pi * f * t) + A3 * np.sin(6 * np.pi * f * t + 0.3))
        h = dg.spectrum(t, p, f, 4, packet_cycles=W)
        assert abs(h[0] / A1 - 1) < 1e-3 and abs(h[2] / A3 - 1) < 1e-2
        assert h[1] < 1e-3 * A1 and h[3] < 1e-3 * A1


def test_harmonics_of_a_steady_signal():
    """Over a whole number of periods the windowed transform gives the
    amplitude of each sinusoid."""
    f = 2.0
    t = np.linspace(0.0, 5.0 / f, 4001)
    p = 3.0 * np.sin(2 * np.pi * f * t) + 0.5 * np.cos(4 * np.pi * f * t)
    h = dg.harmonics(t, p, f, 3)
    assert abs(h[0] - 3.0) < 1e-4 and abs(h[1] - 0.5) < 1e-4 and h[2] < 1e-4


def test_line_cells_follow_the_propagation_direction():
    """The error line of the oblique Taylor workload: one cell per column (per
    row past 45 degrees), consecutive, 10 units long, every chosen cell within
    half a cell (across the line) of the line through the analytic front."""
    import math
    from paper_1311_3004_amd import inputs
    for theta in (0.0, math.pi / 32, math.pi / 8, math.pi / 4, 3 * math.pi / 8):
        w = inputs.taylor_oblique(10, theta, travel=30.0)
        t = 0.37 * w["t_end"]
        i, j = dg.line_cells(w, t)
        c, s = math.cos(theta), math.sin(theta)
        major = i if abs(c) >= abs(s) else j
        assert np.all(np.diff(major) == 1)
        assert abs(len(major) - 10 * 10 * max(abs(c), abs(s))) <= 1
        fx = w["front0_m"][0] + w["medium"]["c0"] * t * c
        fy = w["front0_m"][1] + w["medium"]["c0"] * t * s
        px, py = (i + 0.5) * w["dx"] - fx, (j + 0.5) * w["dx"] - fy
        across = np.abs(-s * px + c * py) / w["dx"]
        assert np.all(across <= 0.5 * (abs(c) + abs(s)) + 1e-9)
        along = (c * px + s * py) / w["unit_m"]
        assert np.all(np.abs(along) <= 5.0 + 1e-9)


def test_taylor_errors_vanish_on_the_exact_profile_and_see_a_shift():
    """E1 and Einf of eq. (error) are 0 (to rounding) on the analytic profile
    at its own time; a profile one cell behind gives E1 = (total variation of
    the profile, 2a, times the shift in cells, 1) / (sum of |reference| over
    the line's cells), to first order in the shift."""
    from paper_1311_3004_amd import inputs
    w = inputs.taylor_oblique(20, 0.0, travel=10.0, reading="rise")
    R0 = w["state"][0] / w["medium"]["rho0"]
    e1, einf = dg.taylor_errors(w, 0.0, R0)
    assert e1 < 1e-15 and einf < 1e-15
    t = w["dx"] / w["medium"]["c0"]                    # the analytic front one cell ahead
    e1, einf = dg.taylor_errors(w, t, R0)
    i, _ = dg.line_cells(w, t)
    xi = ((i + 0.5) * w["dx"] - w["taylor"]["x0_m"] - w["medium"]["c0"] * t) / w["tanh_unit_m"]
    want = 2.0 / np.sum(np.abs(np.tanh(xi)))
    assert abs(e1 / want - 1.0) < 0.01
    assert 0.05 < einf < 0.2                           # dx / w = 0.11 at the front


def test_packet_workload_geometry():
    """Fixed and moving domains of the packet workload: the same cells per
    wavelength and width, the moving one 24 wavelengths long with its second
    stage at half its length, quarter-wavelength moves, the fixed one
    switching at +6 periods."""
    from paper_1311_3004_amd import inputs
    f = inputs.PACKET_FREQ
    wf = inputs.hifu_packet(eta=40, a=10.0, length_wl=60.0)
    wm = inputs.hifu_packet(eta=40, a=10.0, length_wl=60.0, window_wl=24.0)
    assert wf["ny"] == wm["ny"] == 800 and wf["nx"] == wf["path_cells"] == 2400
    assert wm["nx"] == 960 and wm["path_cells"] == 2400
    assert abs(wf["source"]["stage2_time"] * f - 6.0) < 1e-12
    assert abs(wm["source"]["stage2_time"] * f - 12.0) < 1e-12 and wm["window"]["t1"] == wm["source"]["stage2_time"]
    assert wm["window"]["quantum"] == wm["window"]["check_every"] == 10
    assert abs(wf["t0"] * f + 6.0) < 1e-12 and abs(wf["t_end"] * f - 66.5) < 1e-12


def test_front_shift_measures_a_known_lag_and_ignores_storage_rounding():
    """front_shift on a steepened front (a tanh profile 1.5 cells wide) moved
    by known sub-cell and whole-cell amounts recovers the move to 0.005 cells
    (the bias of linear interpolation on the sampled reference); rounded to
    an 11-bit significand (FP16 storage) it still does to 0.02; a lag beyond
    the scan is reported as None."""
    z = np.arange(3000.0)
    prof = lambda s: 2e6 * np.tanh((1500.0 + s - z) / 1.5) + 1e6 * np.exp(-((z - 1480.0 - s) / 30.0) ** 2)
    ref = prof(0.0)
    for s in (0.37, -1.23, 2.5, 0.0):
        assert abs(dg.front_shift(prof(s), ref, 1500) - s) <= 5e-3
        q = np.float16(prof(s) / 4e6).astype(np.float64) * 4e6
        assert abs(dg.front_shift(q, ref, 1500) - s) <= 2e-2
    assert dg.front_shift(prof(12.0), ref, 1500, max_shift=8.0) is None
