"""Pins of the 3-D oracle (the paper's equations in three dimensions, Sec. 5:
three sweeps, four conserved components), all on the CPU."""
import numpy as np
import pytest

from oracle import oracle3d as o3


@pytest.fixture(scope="module", autouse=True)
def _built():
    o3.build()


def flux4(beta, q):          # written out independently of the C code
    R, Mn, Mt1, Mt2 = q
    r = 1.0 + R
    return np.array([Mn, (Mn / r) ** 2 + R + (beta - 1) * R * R, Mn * Mt1 / r ** 2, Mn * Mt2 / r ** 2])

def test_roe_property_four_components():
    """The 4-component Roe decomposition: its fluctuations add up to the flux
    difference written out here independently (mass Mn, momentum un^2 + phi,
    tangential un ut1, un ut2), and its waves to the jump, for 2000 random
    state pairs and beta in [1, 5]."""
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(2000):
        beta = rng.uniform(1, 5)
        qL = rng.uniform(-0.05, 0.05, 4); qR = qL + rng.uniform(-0.02, 0.02, 4)
        ok, s, al, W, amdq, apdq = o3.roe(beta, qL, qR)
        assert ok
        df = flux4(beta, qR) - flux4(beta, qL)
        err = np.max(np.abs(amdq + apdq - df)) / max(np.max(np.abs(df)), 1e-300)
        worst = max(worst, err)
        assert np.max(np.abs(W.sum(axis=0) - (qR - qL))) < 1e-15
    assert worst < 2e-12

def _pulse(n, rng, amp=0.02):
    x = np.arange(n) + 0.5
    return amp * np.exp(-((x - n / 2) / (n / 8)) ** 2) * (1 + 0.1 * rng.uniform(-1, 1, n))

def test_plane_waves_reduce_to_the_2d_oracle(orc):
    """A state that varies along one axis only (two periodic axes of 4 cells,
    extrapolating and reflecting ends, viscous, a tangential momentum on a
    second axis) must evolve exactly as the 2-D oracle's run of the same line,
    whichever axis it lies along; the third momentum stays exactly zero."""
    rng = np.random.default_rng(7)
    n, beta, delta = 48, 4.2, 0.01
    R = _pulse(n, rng); M = R * 0.7 + _pulse(n, rng, 0.003); T = _pulse(n, rng, 0.004)
    # 2-D oracle along x: (R, M, N) over 48 x 4, periodic y
    p2 = orc.make_params(n, 4, beta, delta, bc=("extrap0", "reflect", "periodic", "periodic"), fixed_dt=True)
    A = lambda v: np.tile(v[None, :], (4, 1))
    R2, M2, N2, i2 = orc.run(p2, A(R), A(M), A(T), 30, dt=0.8)
    assert i2["status"] == 0
    for axis in range(3):
        shape = [4, 4, 4]; shape[2 - axis] = n      # arrays are [z][y][x]
        bc = ["periodic"] * 6; bc[2 * axis] = "extrap0"; bc[2 * axis + 1] = "reflect"
        p3 = o3.make_params(shape[2], shape[1], shape[0], beta, delta, bc=bc, fixed_dt=True)
        def F(v):
            sl = [None, None, None]; sl[2 - axis] = slice(None)
            return np.broadcast_to(v[tuple(sl)], shape).copy()
        Z = np.zeros(shape)
        Q = [F(R), Z.copy(), Z.copy(), Z.copy()]
        Q[1 + axis] = F(M)
        t_comp = 1 + (axis + 1) % 3           # put the tangential momentum on another axis
        Q[t_comp] = F(T)
        Q3, i3 = o3.run(p3, Q, 30, dt=0.8)
        assert i3["status"] == 0
        sel = [0, 0, 0]; sel[2 - axis] = slice(None)
        got = [Q3[0][tuple(sel)], Q3[1 + axis][tuple(sel)], Q3[t_comp][tuple(sel)]]
        want = [R2[0], M2[0], N2[0]]
        err = max(np.max(np.abs(g - w)) for g, w in zip(got, want)) / np.max(np.abs(R))
        other = [c for c in (1, 2, 3) if c not in (1 + axis, t_comp)][0]
        assert err < 1e-13 and np.max(np.abs(Q3[other])) == 0.0

def test_conservation_periodic_box():
    """Telescoping fluxes and a Laplacian summing to zero: on a periodic box
    the sums of R, M1, M2, M3 are constant to rounding over 25 steps."""
    rng = np.random.default_rng(9)
    nx, ny, nz = 14, 12, 10
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    R = 0.02 * np.sin(2 * np.pi * x / nx) * np.cos(2 * np.pi * y / ny) + 0.01 * np.sin(2 * np.pi * z / nz) + 0.002 * rng.uniform(-1, 1, (nz, ny, nx))
    Q = [R, 0.5 * R + 0.001 * rng.uniform(-1, 1, R.shape), 0.001 * rng.uniform(-1, 1, R.shape), -0.3 * R]
    p = o3.make_params(nx, ny, nz, 4.0, 0.02, bc=("periodic",) * 6)
    Q2, info = o3.run(p, Q, 25)
    assert info["status"] == 0 and info["steps"] == 25
    for a, b in zip(Q, Q2):
        rel = abs(a.sum() - b.sum()) / np.abs(a).sum()
        assert rel < 1e-13


def test_linear_diagonal_mode_converges():
    """Linear small-amplitude limit along the box diagonal, k = 2 pi/L (1, 1, 1):
    dR/dt + div m = 0, dm/dt + grad R = delta~ lap m for the mode e^{i k.x}
    solved exactly (4 x 4 matrix exponential), R(0) = eps cos(k.x) as cell
    averages, m(0) = 0, fixed dt = 0.45, a quarter box length of travel; the
    mean error of R converges at order > 1.7 (16, 32, 64 cells per side).  (A
    start with a shear part converges at order ~1 along diagonals: the
    splitting error of Godunov splitting, which the paper's method has.)"""
    from scipy.linalg import expm
    eps, beta, dtil_unit, dt = 1e-6, 4.0, 5e-4, 0.45
    errs = []
    for L in (16, 32, 64):
        k = 2 * np.pi / L * np.array([1.0, 1.0, 1.0])
        delta = dtil_unit * L
        A = np.zeros((4, 4), dtype=complex)
        A[0, 1:] = -1j * k
        A[1:, 0] = -1j * k
        A[1:, 1:] = -(delta * (k @ k)) * np.eye(3)
        z, y, x = np.meshgrid(*(np.arange(L) + 0.5,) * 3, indexing="ij")
        sinc = np.prod([np.sinc(kc / (2 * np.pi)) for kc in k])   # cell averages
        ph = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
        Z = np.zeros((L, L, L))
        Q = [eps * sinc * np.real(ph), Z, Z, Z]
        p = o3.make_params(L, L, L, beta, delta, bc=("periodic",) * 6, fixed_dt=True)
        Q, info = o3.run(p, Q, int(round(0.25 * L / dt)), dt=dt)
        assert info["status"] == 0
        qt = expm(A * info["t"]) @ np.array([1.0, 0, 0, 0], dtype=complex)
        ex = eps * sinc * np.real(qt[0] * ph)
        errs.append(np.mean(np.abs(Q[0] - ex)) / np.mean(np.abs(ex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.7) and errs[-1] < 2e-2
