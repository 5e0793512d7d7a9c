"""The 3-D step through its C ABI against the 3-D FP64 oracle: a ragged grid
with all three side kinds, a seeded pulse with momentum in every component,
fixed and adaptive time steps, FP64 and FP32.  Tolerances relative to the
peak |R|: FP64 1e-12 (fixed dt) / 1e-10 (adaptive), FP32 2e-6."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MED = {"c0": 1500.0, "rho0": 1000.0, "beta": 3.5, "delta": 4.3e-6}
DX = 1e-4
BC = ("extrap0", "reflect", "periodic", "periodic", "reflect", "extrap0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _state(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    a = 2e6 / (MED["rho0"] * MED["c0"] ** 2)
    sig = max(3.0, min(nx, ny, nz) / 12.0)
    R = a * np.exp(-((x - 0.45 * nx) ** 2 + (y - 0.5 * ny) ** 2 + (z - 0.4 * nz) ** 2) / (2 * sig ** 2))
    R = R + 0.01 * a * rng.uniform(-1, 1, R.shape)
    M = [c * R for c in (0.3, -0.2, 0.25)]
    return R, M


def _run_pair(precision, steps, fixed, dt_cells=0.6, shape=(20, 14, 10), seed=3, bc=BC, first_dt_cells=None):
    """first_dt_cells (adaptive runs): the first attempt's dt in cells / c0
    instead of the dry pass's."""
    from paper_1311_3004_amd import fvna3d as f3
    from oracle import oracle3d as o3
    nx, ny, nz = shape
    R, M = _state(nx, ny, nz, seed)
    rho0, c0 = MED["rho0"], MED["c0"]
    if not fixed and first_dt_cells is not None:
        dt_cells = first_dt_cells
    dt_si = dt_cells * DX / c0 if (fixed or first_dt_cells is not None) else 0.0
    p = f3.make_params(nx, ny, nz, DX, MED, bc=bc, precision=precision, fixed_dt=fixed, dt0=dt_si)
    s = f3.Sim3(p)
    s.fvna3_set_state(R * rho0, *[m * rho0 * c0 for m in M])
    s.fvna3_step(steps)
    g = s.fvna3_get_state()
    st = s.fvna3_get_stats()
    s.fvna3_destroy()
    g = (g[0] / rho0,) + tuple(m / (rho0 * c0) for m in g[1:])
    po = o3.make_params(nx, ny, nz, MED["beta"], MED["delta"] / (c0 * DX), bc=bc, fixed_dt=fixed)
    o, info = o3.run(po, [R] + M, steps, dt=dt_cells if (fixed or first_dt_cells is not None) else 0.0)
    assert info["status"] == 0 and st["steps"] == steps
    err = max(np.max(np.abs(a - b)) for a, b in zip(g, o)) / np.max(np.abs(o[0]))
    return err, st, info


@pytest.mark.parametrize("precision,fixed,tol", [("f64", True, 1e-12), ("f64", False, 1e-10), ("f32", True, 2e-6)])
def test_3d_step_vs_oracle(precision, fixed, tol):
    _say(f"case: 3-D 20x14x10 {precision} {'fixed' if fixed else 'adaptive'} dt, 12 steps")
    err, st, info = _run_pair(precision, 12, fixed)
    _say(f"  max rel err {err:.3e}")
    assert err <= tol
    if not fixed:
        assert abs(st["t"] * MED["c0"] / DX - info["t"]) <= 1e-12 * info["t"]


@pytest.mark.parametrize("precision,fixed,tol", [("f64", True, 1e-12), ("f64", False, 1e-10),
                                                 ("f32", True, 2e-6), ("f32", False, 2e-6)])
def test_3d_step_vs_oracle_large(precision, fixed, tol):
    """128 x 96 x 96 = 1.18 M cells: many wavefronts per sweep and plane, every
    side kind, FP32 also with the adaptive time step."""
    shape = (128, 96, 96)
    _say(f"case: 3-D {shape} {precision} {'fixed' if fixed else 'adaptive'} dt, 2 steps")
    err, st, info = _run_pair(precision, 2, fixed, shape=shape, seed=21)
    _say(f"  max rel err {err:.3e}")
    assert err <= tol
    if not fixed:
        rel_t = 1e-12 if precision == "f64" else 1e-7
        assert abs(st["t"] * MED["c0"] / DX - info["t"]) <= rel_t * info["t"]


BC_PERIODIC_X = ("periodic", "periodic", "reflect", "extrap0", "periodic", "periodic")


@pytest.mark.parametrize("shape", [(76, 18, 7), (140, 12, 7)])
@pytest.mark.parametrize("precision,fixed,tol", [("f64", True, 1e-12), ("f32", False, 2e-6)])
def test_3d_packed_tail_vs_oracle(shape, precision, fixed, tol):
    """The x1-x2 sweep's packed tail: the last nx mod 60 columns (16 and 20)
    of three and two planes per wavefront, 7 planes so that the last tail
    wavefront has idle segments, periodic x1 (the tail's right halo wraps to
    the first columns) and x3, reflecting / extrapolating x2."""
    _say(f"case: 3-D packed tail {shape} {precision} {'fixed' if fixed else 'adaptive'} dt, 8 steps")
    err, st, info = _run_pair(precision, 8, fixed, shape=shape, seed=7, bc=BC_PERIODIC_X)
    _say(f"  max rel err {err:.3e}")
    assert err <= tol
    if not fixed:
        assert abs(st["t"] * MED["c0"] / DX - info["t"]) <= 1e-7 * info["t"]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-10), ("f32", 2e-6)])
def test_3d_rejected_first_step_is_redone_from_the_same_state(precision, tol):
    """A first dt three times the CFL limit: the attempt is rejected, redone
    from the untouched state with dt nu_W / nu, and the run goes on as in the
    oracle (the state's density and momenta live in different buffers, and a
    rejected attempt writes neither of them)."""
    _say(f"case: 3-D rejected first step, {precision}")
    err, st, info = _run_pair(precision, 12, False, first_dt_cells=3.0)
    assert info["rejected"] == 1 and st["rejected"] == 1
    assert err <= tol, err


def test_3d_refuses_bad_parameters():
    from paper_1311_3004_amd import fvna, fvna3d as f3
    for bc in (("taylor",) * 6, ("periodic", "extrap0") + ("extrap0",) * 4):
        p = f3.make_params(8, 8, 8, DX, MED, bc=bc)
        with pytest.raises(fvna.FvnaError):
            f3.Sim3(p)
    with pytest.raises(fvna.FvnaError):
        f3.Sim3(f3.make_params(3, 8, 8, DX, MED))


def test_3d_reports_a_nonhyperbolic_state():
    """A state outside the model's hyperbolic region (velocity twice the
    sound speed) is refused when the first step is computed from it, with
    FVNA_E_NONHYPERBOLIC; the context stays usable for a valid state."""
    from paper_1311_3004_amd import fvna, fvna3d as f3
    nx, ny, nz = 12, 10, 8
    s = f3.Sim3(f3.make_params(nx, ny, nz, DX, MED, bc=BC))
    Z = np.zeros((nz, ny, nx))
    R = Z + 0.01
    with pytest.raises(fvna.FvnaError) as e:
        s.fvna3_set_state(R * MED["rho0"], (1 + R) * 2.0 * MED["rho0"] * MED["c0"], Z, Z)
    assert e.value.status == fvna.E_NONHYPERBOLIC
    R, M = _state(nx, ny, nz, 11)
    s.fvna3_set_state(R * MED["rho0"], *[m * MED["rho0"] * MED["c0"] for m in M])
    s.fvna3_step(3)
    assert s.fvna3_get_stats()["steps"] == 3
    s.fvna3_destroy()


@pytest.fixture(scope="module")
def bench3d_oracle():
    """The 3-D benchmark workload (256^3 Gaussian pulse, sigma 8 cells, 2 MPa,
    0.5% noise with seed 5, water, extrapolating sides) and one fixed-dt step
    of the FP64 oracle on it (about 20 s on one host core)."""
    from oracle import oracle3d as o3
    from paper_1311_3004_amd.inputs import WATER
    n = 256
    med = dict(WATER)
    rng = np.random.default_rng(5)
    c = (np.arange(n) + 0.5 - n / 2) ** 2
    a = 2e6 / (med["rho0"] * med["c0"] ** 2)
    R = a * np.exp(-(c[:, None, None] + c[None, :, None] + c[None, None, :]) / (2 * 8.0 ** 2))
    R += 0.005 * a * rng.uniform(-1, 1, R.shape)
    Z = np.zeros_like(R)
    _say("case: 3-D 256^3 benchmark workload, oracle FP64, 1 fixed-dt step")
    po = o3.make_params(n, n, n, med["beta"], med["delta"] / (med["c0"] * 1e-4), bc=("extrap0",) * 6,
                        fixed_dt=True)
    o, info = o3.run(po, [R, Z, Z, Z], 1, dt=0.6)
    assert info["status"] == 0
    return med, R, o


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_3d_benchmark_size_one_step_vs_oracle(bench3d_oracle, precision, tol):
    """The 256^3 workload bench.py times, in the launch plan it times (four
    60-column strips and a three-plane packed tail, 43-row segments over
    several rounds, the x3 sweep and the source in one round of z-segments):
    one fixed-dt step, every cell against the oracle."""
    from paper_1311_3004_amd import fvna3d as f3
    med, R, o = bench3d_oracle
    n = R.shape[0]
    rho0, c0 = med["rho0"], med["c0"]
    _say(f"case: 3-D 256^3 benchmark workload {precision}, 1 fixed-dt step")
    p = f3.make_params(n, n, n, 1e-4, med, bc=("extrap0",) * 6, precision=precision, fixed_dt=True,
                       dt0=0.6 * 1e-4 / c0)
    s = f3.Sim3(p)
    Z = np.zeros_like(R)
    s.fvna3_set_state(R * rho0, Z, Z, Z)
    s.fvna3_step(1)
    g = s.fvna3_get_state()
    st = s.fvna3_get_stats()
    s.fvna3_destroy()
    assert st["steps"] == 1 and st["status"] == 0
    g = (g[0] / rho0,) + tuple(m / (rho0 * c0) for m in g[1:])
    err = max(np.max(np.abs(a - b)) for a, b in zip(g, o)) / np.max(np.abs(o[0]))
    _say(f"  max rel err {err:.3e}")
    assert err <= tol
