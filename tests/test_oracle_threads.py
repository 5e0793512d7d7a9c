"""The oracle's OpenMP rows give bitwise the serial result (CPU).

The CPU baseline is timed on one thread and on all host cores; that is only
the same oracle if the threaded run computes exactly what the serial run does.
"""
import numpy as np
import pytest

from common import dimless_state, oracle_params, pulse_workload


def _cases():
    from paper_1311_3004_amd import inputs
    yield "pulse, reflect/periodic", pulse_workload(70, 46, ("reflect", "reflect", "periodic", "periodic"), seed=3), {}
    yield "pulse, extrap/reflect", pulse_workload(53, 61, ("extrap0", "extrap0", "reflect", "extrap0"), seed=4), {}
    src = {"freq": 1e6, "p_surface": 2e5, "focal_length": 2e-3, "aperture": 0.8e-3, "ramp_cycles": 1.0}
    yield "axisymmetric focused source", pulse_workload(64, 48, ("source", "extrap0", "reflect", "extrap0"),
                                                        geometry="axisym", seed=5, dx=2e-5, source=src), {}
    yield "taylor sides", inputs.taylor_oblique(5, 0.3, travel=6.0, margin=3.0), {}


@pytest.mark.parametrize("threads", [3, 8])
def test_threads_give_the_serial_result_bitwise(orc, threads):
    for name, w, over in _cases():
        p = oracle_params(orc, w, **over)
        R, M, N = dimless_state(w)
        t0 = w.get("t0", 0.0) * w["medium"]["c0"] / w["dx"]
        orc.set_threads(1)
        a = orc.run(p, R, M, N, 7, t=t0, want_hist=True)
        orc.set_threads(threads)
        try:
            b = orc.run(p, R, M, N, 7, t=t0, want_hist=True)
        finally:
            orc.set_threads(1)
        assert a[3]["status"] == 0 and b[3]["status"] == 0, name
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y), name
        assert np.array_equal(a[3]["nu_hist"], b[3]["nu_hist"]), name
        assert a[3]["t"] == b[3]["t"] and a[3]["dt_next"] == b[3]["dt_next"], name
