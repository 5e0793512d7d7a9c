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
