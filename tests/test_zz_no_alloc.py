"""fvna_sums_noalloc (the sums entry point for callers that cannot allocate)
against fvna_sums on the same state: two calls in a row through the C ABI,
the second on a smaller grid, both bitwise equal to the context's own sums."""
import sys

import numpy as np
import pytest

from common import pulse_workload


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.gpu
def test_sums_noalloc_matches_fvna_sums_twice_second_smaller():
    import torch
    from paper_1311_3004_amd import fvna

    cases = [(1100, 700, "f64", 3), (300, 180, "f32", 2)]
    for nx, ny, prec, steps in cases:
        _say(f"case: sums_noalloc {nx}x{ny} {prec} after {steps} steps")
        w = pulse_workload(nx, ny, ("extrap0",) * 4, seed=nx)
        s = fvna.sim_from_workload(w, precision=prec, fixed_dt=True, dt0=2e-8)
        s.fvna_step(steps)
        ref = s.fvna_sums()
        st = s.fvna_get_stats()
        assert st["steps"] == steps and st["rejected"] == 0
        # the current state is in buffer A after an even number of accepted
        # steps (no moves), else in B
        cur = s.buf_a if st["steps"] % 2 == 0 else s.buf_b
        out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda:0")
        fvna.fvna_sums_noalloc(s.params, cur, out, stream=s.stream)
        s.stream.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (got, ref)
        # and both are the sums of the exported state (independent check)
        rp, mx, my = s.fvna_get_state()
        for g, f in zip(got, (rp, mx, my)):
            exact = float(np.sum(f, dtype=np.float64))
            scale = float(np.sum(np.abs(f))) + 1e-300
            assert abs(g - exact) <= 1e-12 * scale, (g, exact)
        s.fvna_destroy()


@pytest.mark.gpu
def test_sums_noalloc_rejects_bad_arguments():
    import torch
    from paper_1311_3004_amd import fvna

    w = pulse_workload(64, 64, ("extrap0",) * 4)
    p = fvna.make_params(64, 64, 1e-4, w["medium"], precision="f64")
    out = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    st = fvna.lib.fvna_sums_noalloc(fvna.ctypes.byref(p), None, None,
                                    fvna.ctypes.c_void_p(out.data_ptr()))
    assert st == fvna.E_INVALID
    bad = fvna.make_params(3, 64, 1e-4, w["medium"], precision="f64")
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda:0")
    st = fvna.lib.fvna_sums_noalloc(fvna.ctypes.byref(bad), fvna.ctypes.c_void_p(buf.data_ptr()), None,
                                    fvna.ctypes.c_void_p(out.data_ptr()))
    assert st == fvna.E_INVALID and "at least 4" in fvna.last_error()
