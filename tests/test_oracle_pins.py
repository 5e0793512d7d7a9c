"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these tests re-types an oracle formula and compares it with itself:
each checks a property that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle would break.
"""
import math

import numpy as np
import pytest

BETA = 3.5


def paper_flux(beta, q):
    """x1 flux of eq. adim:q, ambient pressure removed, in perturbation form."""
    R, M, N = q
    q1 = 1.0 + R
    return np.array([M, M * M / (q1 * q1) + R + (beta - 1.0) * R * R, M * N / (q1 * q1)])


def paper_roe_matrix(beta, qL, qR):
    """A-hat of Sec. 3.2 built from its printed entries."""
    zL = np.array([1 + qL[0], qL[1] / (1 + qL[0]), qL[2] / (1 + qL[0])])
    zR = np.array([1 + qR[0], qR[1] / (1 + qR[0]), qR[2] / (1 + qR[0])])
    Z = 0.5 * (zL + zR)
    Phi = 1 + 2 * (beta - 1) * (0.5 * (qL[0] + qR[0]))
    return np.array([[0.0, 1.0, 0.0],
                     [-2 * Z[1] ** 2 / Z[0] + Phi, 2 * Z[1] / Z[0], 0.0],
                     [-2 * Z[1] * Z[2] / Z[0], Z[2] / Z[0], Z[1] / Z[0]]])


def random_pairs(rng, n, amp, near=None):
    qL = rng.uniform(-amp, amp, size=(n, 3))
    if near is None:
        qR = rng.uniform(-amp, amp, size=(n, 3))
    else:
        qR = qL + rng.uniform(-near, near, size=(n, 3))
    return qL, qR


# -- P1: Roe property, eq. RoeCond --------------------------------------------

@pytest.mark.parametrize("amp,near", [(0.05, None), (1e-3, None), (1e-3, 1e-7), (0.1, 1e-4)])
def test_roe_property_flux_difference(orc, amp, near):
    rng = np.random.default_rng(11)
    qL, qR = random_pairs(rng, 400, amp, near)
    for a, b in zip(qL, qR):
        d = orc.roe(BETA, a, b)
        assert d is not None
        df = paper_flux(BETA, b) - paper_flux(BETA, a)
        total = d["amdq"] + d["apdq"]              # = sum_p s^p W^p = A-hat dQ
        scale = np.max(np.abs(df)) + 1e-300
        # the reference difference itself carries the rounding of each flux
        fscale = max(np.max(np.abs(paper_flux(BETA, a))), np.max(np.abs(paper_flux(BETA, b))))
        assert np.max(np.abs(total - df)) <= 2e-13 * scale + 4e-16 * fscale
        # waves add up to the jump
        assert np.allclose(d["W"].sum(axis=0), b - a, rtol=0, atol=1e-15 * np.max(np.abs(b - a)) + 1e-300)


# -- P2: eigen-structure against the printed matrix and eqs. lambda1-3 ---------

def test_eigenpairs_of_printed_matrix(orc):
    rng = np.random.default_rng(12)
    qL, qR = random_pairs(rng, 300, 0.05)
    for a, b in zip(qL, qR):
        d = orc.roe(BETA, a, b)
        A = paper_roe_matrix(BETA, a, b)
        ev = np.sort(np.linalg.eigvals(A).real)
        assert np.allclose(np.sort(d["s"]), ev, rtol=0, atol=1e-14)
        for p in range(3):
            r = d["r"][p]
            res = A @ r - d["s"][p] * r
            assert np.max(np.abs(res)) <= 1e-14 * (1 + np.max(np.abs(r)))


def test_near_equilibrium_speeds(orc):
    """eqs. lambda:p1-p3: s = (u +- c)/c0, u/c0 with c = c0 (1 + (beta-1) rho'/rho0),
    up to O(eps^2)."""
    rng = np.random.default_rng(13)
    for eps in (1e-3, 1e-4):
        for _ in range(50):
            R = rng.uniform(-eps, eps)
            u = rng.uniform(-eps, eps)
            q = np.array([R, (1 + R) * u, (1 + R) * rng.uniform(-eps, eps)])
            d = orc.roe(BETA, q, q)
            c = 1 + R * (BETA - 1)
            assert abs(d["s"][0] - (u + c)) < 10 * eps ** 2
            assert abs(d["s"][1] - (u - c)) < 10 * eps ** 2
            assert abs(d["s"][2] - u) < 10 * eps ** 2


# -- P3: consistency (property (i) of Sec. 3.2) --------------------------------

def test_roe_matrix_tends_to_jacobian(orc):
    rng = np.random.default_rng(14)
    h = 1e-6
    for _ in range(50):
        q = rng.uniform(-0.05, 0.05, 3)
        J = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3); e[k] = h
            J[:, k] = (paper_flux(BETA, q + e) - paper_flux(BETA, q - e)) / (2 * h)
        d = orc.roe(BETA, q, q)
        # oracle's A-hat rebuilt from its eigen-decomposition
        Rm = d["r"].T
        A = Rm @ np.diag(d["s"]) @ np.linalg.inv(Rm)
        assert np.max(np.abs(A - J)) < 1e-8


# -- P4: hyperbolicity region S(rho/rho0) --------------------------------------

def test_hyperbolicity_region_matches_paper_criterion(orc):
    beta = 4.8
    mism = 0
    checked = 0
    for rho in np.linspace(0.05, 2.0, 79):
        for u in np.linspace(-3.0, 3.0, 121):
            S = max(0.0, (1 + 2 * (beta - 1) * (rho - 1)) / (2 * rho - 1) * rho ** 2) \
                if abs(2 * rho - 1) > 1e-12 else None
            if S is None or abs(u * u - S) < 1e-6 or u == 0.0:
                continue
            ok_paper = (rho < 0.5 and u * u > S) or (rho > 0.5 and u * u < S)
            q = np.array([rho - 1, rho * u, 0.0])
            ok_orc = orc.roe(beta, q, q) is not None
            checked += 1
            mism += ok_paper != ok_orc
    assert checked > 5000
    assert mism == 0


# -- P5: MC limiter values -------------------------------------------------------

@pytest.mark.parametrize("theta,phi", [(-1, 0), (0, 0), (0.25, 0.5), (0.5, 0.75), (1, 1),
                                       (2, 1.5), (3, 2), (10, 2), (-1e9, 0), (1e9, 2)])
def test_mc_limiter_table(orc, theta, phi):
    assert orc.mc(theta) == phi


# -- P14: one step of an isolated jump is a Godunov step ----------------------

def test_isolated_jump_first_step_is_godunov(orc):
    nx, ny = 24, 4
    qa = np.array([2e-3, 1.5e-3, -4e-4])
    qb = np.array([-1e-3, 5e-4, 7e-4])
    R = np.empty((ny, nx)); M = np.empty((ny, nx)); N = np.empty((ny, nx))
    R[:, :12], M[:, :12], N[:, :12] = qa
    R[:, 12:], M[:, 12:], N[:, 12:] = qb
    dt = 0.4
    p = orc.make_params(nx, ny, BETA, 0.0, bc=("extrap0", "extrap0", "periodic", "periodic"),
                        fixed_dt=True)
    R1, M1, N1, info = orc.run(p, R, M, N, 1, dt=dt)
    assert info["status"] == 0
    # independent decomposition with numpy: eigenvectors of the printed matrix
    A = paper_roe_matrix(BETA, qa, qb)
    lam, V = np.linalg.eig(A)
    lam, V = lam.real, V.real
    alpha = np.linalg.solve(V, qb - qa)
    amdq = sum(min(lam[p], 0) * alpha[p] * V[:, p] for p in range(3))
    apdq = sum(max(lam[p], 0) * alpha[p] * V[:, p] for p in range(3))
    got = np.stack([R1, M1, N1], axis=-1)
    exp = np.stack([R, M, N], axis=-1).copy()
    exp[:, 11] = qa - dt * amdq
    exp[:, 12] = qb - dt * apdq
    assert np.max(np.abs(got - exp)) <= 1e-15 * 4


# -- P9: conservation on a doubly periodic grid --------------------------------

@pytest.mark.parametrize("delta", [0.0, 0.05])
def test_conservation_periodic(orc, delta):
    nx, ny = 40, 36
    rng = np.random.default_rng(15)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    R = 3e-3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.01) + 2e-4 * rng.uniform(-1, 1, (ny, nx))
    M = 1e-3 * np.sin(2 * np.pi * X) + 1e-4 * rng.uniform(-1, 1, (ny, nx))
    N = 1e-3 * np.cos(2 * np.pi * Y)
    p = orc.make_params(nx, ny, BETA, delta, bc=("periodic",) * 4)
    s0 = np.array([R.sum(), M.sum(), N.sum()])
    R1, M1, N1, info = orc.run(p, R, M, N, 60)
    assert info["status"] == 0
    s1 = np.array([R1.sum(), M1.sum(), N1.sum()])
    scale = np.array([np.abs(R).sum(), np.abs(M).sum(), np.abs(N).sum()])
    assert np.all(np.abs(s1 - s0) <= 1e-13 * scale)
    # and the state really changed
    assert np.max(np.abs(R1 - R)) > 1e-4


# -- P10: mirror symmetry ------------------------------------------------------

@pytest.mark.parametrize("bcx", ["extrap0", "reflect"])
def test_mirror_symmetry_x_and_y(orc, bcx):
    nx, ny = 48, 40
    x = np.arange(nx) + 0.5 - nx / 2          # centre on a cell corner
    y = np.arange(ny) + 0.5 - ny / 2
    X, Y = np.meshgrid(x, y)
    R = 5e-3 * np.exp(-(X ** 2 + Y ** 2) / (2 * 4.0 ** 2))
    M = np.zeros_like(R); N = np.zeros_like(R)
    p = orc.make_params(nx, ny, BETA, 0.02, bc=(bcx, bcx, bcx, bcx))
    R1, M1, N1, info = orc.run(p, R, M, N, 80)
    assert info["status"] == 0
    peak = np.max(np.abs(R1))
    assert np.max(np.abs(R1 - R1[:, ::-1])) <= 1e-12 * peak
    assert np.max(np.abs(M1 + M1[:, ::-1])) <= 1e-12 * peak
    assert np.max(np.abs(N1 - N1[:, ::-1])) <= 1e-12 * peak
    assert np.max(np.abs(R1 - R1[::-1, :])) <= 1e-12 * peak
    assert np.max(np.abs(M1 - M1[::-1, :])) <= 1e-12 * peak
    assert np.max(np.abs(N1 + N1[::-1, :])) <= 1e-12 * peak
    assert np.max(np.abs(M1)) > 1e-5   # the pulse did spread


# -- P6: linear small-amplitude limit, exact per Fourier mode -------------------

def linear_mode_exact(n, kx_m, ky_m, eps, delta, t):
    """Cell averages of R for the linearised system dR/dt + div m = 0,
    dm/dt + grad R = delta lap m, with R(0) = eps cos(k.x), m(0) = 0, on an
    n x n periodic grid of unit cells."""
    kx = 2 * np.pi * kx_m / n
    ky = 2 * np.pi * ky_m / n
    k2 = kx * kx + ky * ky
    g = delta * k2 / 2
    Om = np.sqrt(k2 - g * g)
    amp = eps * np.exp(-g * t) * (np.cos(Om * t) + g / Om * np.sin(Om * t))
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    sx = np.sinc(kx / (2 * np.pi)) if kx else 1.0   # np.sinc(z) = sin(pi z)/(pi z)
    sy = np.sinc(ky / (2 * np.pi)) if ky else 1.0
    return amp * sx * sy * np.cos(kx * X + ky * Y), sx * sy


@pytest.mark.slow
def test_linear_limit_converges_second_order(orc):
    eps = 1e-9
    errs = []
    ns = [32, 64, 128]
    for n in ns:
        delta = 0.002 * n / 32          # fixed physical diffusivity under refinement
        T = 0.75 * n                    # fixed physical time (0.75 domain lengths)
        dt = 0.45
        steps = int(round(T / dt))
        exact0, fac = linear_mode_exact(n, 2, 1, eps, delta, 0.0)
        R0 = exact0.copy()
        Z = np.zeros_like(R0)
        p = orc.make_params(n, n, BETA, delta, bc=("periodic",) * 4, fixed_dt=True)
        R1, M1, N1, info = orc.run(p, R0, Z, Z, steps, dt=dt)
        assert info["status"] == 0
        ex, _ = linear_mode_exact(n, 2, 1, eps, delta, steps * dt)
        errs.append(np.mean(np.abs(R1 - ex)) / np.mean(np.abs(ex)))
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(2) for i in range(len(errs) - 1)]
    assert errs[-1] < 2e-2
    assert min(rates) > 1.7, (errs, rates)


# -- P7 / P12: Taylor shock-like profile (Sec. 4.1, eq. OurTaylorS, Table 1) ----

def taylor_run(orc, eta, nuw, T=100.0, amp=1e-7, beta=4.0):
    """Thin domain x in [-5, 105] units, eta cells per unit, 4 periodic rows,
    Dirichlet Taylor data on both x ends; run to t = T and return E1, Einf on
    the 10-unit segment centred on the analytic front (eq. error), and the
    standard deviation of nu."""
    nx, ny = int(round(110 * eta)), 4
    x0 = 5.0 * eta
    p = orc.make_params(nx, ny, beta, amp * beta * eta, bc=("taylor", "taylor", "periodic", "periodic"),
                        cfl_target=nuw, taylor={"amp": amp, "width": float(eta), "x0": x0})
    x = np.arange(nx) + 0.5
    R = np.broadcast_to(-amp * np.tanh((x - x0) / eta), (ny, nx)).copy()
    M = R.copy()
    N = np.zeros_like(R)
    tend = T * eta
    t, dt, hist = 0.0, 0.0, []
    # run in chunks while a whole chunk fits, then one step at a time
    while True:
        R2, M2, N2, info = orc.run(p, R, M, N, 100, t=t, dt=dt, want_hist=True)
        if info["t"] >= tend:
            break
        R, M, N, t, dt = R2, M2, N2, info["t"], info["dt_next"]
        hist += list(info["nu_hist"])
    while t + dt <= tend:
        R, M, N, info = orc.run(p, R, M, N, 1, t=t, dt=dt, want_hist=True)
        t, dt = info["t"], info["dt_next"]
        hist += list(info["nu_hist"])
    p.fixed_dt = 1
    R, M, N, info = orc.run(p, R, M, N, 1, t=t, dt=tend - t)
    t = info["t"]
    sel = np.abs(x - (x0 + tend)) <= 5 * eta
    ref = -amp * np.tanh((x[sel] - x0 - t) / eta)
    num = R[0, sel]
    e1 = np.sum(np.abs(num - ref)) / np.sum(np.abs(ref))
    einf = np.max(np.abs(num - ref)) / np.max(np.abs(ref))
    return e1, einf, float(np.std(hist))


@pytest.mark.slow
def test_taylor_shock_table1_band(orc):
    """Table 1, theta_T = 0: E1 convergence rates 1.63..2.00 and E1 at the
    finest mesh 2.36e-5 (best) .. 2.91e-4 (worst); nu std below 1e-8.
    The mesh parameter is read as cells per 10%-90% rise of the step, which is
    2.197 tanh units, the paper's eta read as cells per 10-90% rise, so the paper's eta = 82 is 37.3 cells per
    tanh unit here; E1 there is extrapolated from eta = 5, 10, 20 with the
    measured rate and must fall inside the printed band (factor 2 margin)."""
    etas = [5, 10, 20]
    for nuw in (0.6, 0.99):
        res = [taylor_run(orc, e, nuw) for e in etas]
        e1 = np.array([r[0] for r in res])
        assert np.all(np.diff(e1) < 0)
        rate = -np.polyfit(np.log(etas), np.log(e1), 1)[0]
        assert 1.5 < rate < 2.5, rate
        e82 = e1[-1] * (20.0 / (82.0 / 2.197)) ** rate
        assert 2.36e-5 / 2 < e82 < 2.91e-4 * 2, e82
        for r in res:
            assert r[2] < 1e-8


# -- P13: captured plane shock of the taylor-step workload ---------------------

@pytest.mark.slow
def test_taylor_step_front_position(orc):
    """A symmetric jump R = +-a, M = R moves at the Rankine-Hugoniot speed
    c0 (1 + O(a^2)); after 200 adaptive steps the front (R = 0 crossing,
    averaged over rows) sits at x0 + t within half a cell."""
    from paper_1311_3004_amd import inputs
    w = inputs.c1_taylor_fp64()
    med = w["medium"]
    p = orc.make_params_si(w["nx"], w["ny"], w["dx"], med["c0"], med["rho0"], med["beta"],
                           med["delta"], bc=w["bc"])
    rp, mx, my = w["state"]
    R = rp / med["rho0"]; M = mx / (med["rho0"] * med["c0"]); N = my / (med["rho0"] * med["c0"])
    R1, M1, N1, info = orc.run(p, R, M, N, w["steps"], want_hist=True)
    assert info["status"] == 0 and info["rejected"] == 0
    fronts = []
    for row in R1:
        k = np.nonzero((row[:-1] > 0) & (row[1:] <= 0))[0][-1]
        fronts.append(k + 0.5 + row[k] / (row[k] - row[k + 1]))
    assert abs(np.mean(fronts) - (64.0 + info["t"])) < 0.5
    assert abs(info["nu_mean"] - 0.9) < 1e-3


# -- Axisymmetric source terms: exact Bessel modes ------------------------------

def _axisym_mode_run(orc, n, which, dt=0.45):
    """Uniform in z (4 periodic columns), n cells in r, wall at r = n where
    J1(k n) = 0 (reflecting side: zero normal momentum, even density).
    which = 'shear': M = eps J0(k r) e^{-delta k^2 t}, R = N = 0 -- an exact solution
    of the full axisymmetric system (tests delta (d2/dr2 + (1/r) d/dr) of u).
    which = 'radial': R = eps J0(k r) A(t), N = eps J1(k r) B(t) -- exact for the
    linearised system (tests -N/r in the mass equation and the cylindrical viscous
    terms of v, including -v/r^2); A, B solve the same 2x2 system as a plane mode."""
    from scipy.special import j0, j1, jn_zeros
    eps = 1e-9 if which == "radial" else 1e-6
    kL = jn_zeros(1, 2)[1] if which == "radial" else jn_zeros(1, 1)[0]
    k = kL / n
    delta = 0.02 * n / 32            # fixed physical diffusivity under refinement
    T = 0.6 * n                      # fixed physical time
    steps = int(round(T / dt))
    dt = T / steps
    r = np.arange(n) + 0.5
    nz = 4
    Z = np.zeros((n, nz))
    if which == "shear":
        M0 = np.repeat((eps * j0(k * r))[:, None], nz, axis=1)
        R0, N0 = Z.copy(), Z.copy()
    else:
        R0 = np.repeat((eps * j0(k * r))[:, None], nz, axis=1)
        M0, N0 = Z.copy(), Z.copy()
    p = orc.make_params(nz, n, 3.5, delta, bc=("periodic", "periodic", "reflect", "reflect"),
                        geometry="axisym", fixed_dt=True)
    R1, M1, N1, info = orc.run(p, R0, M0, N0, steps, dt=dt)
    assert info["status"] == 0
    t = steps * dt
    if which == "shear":
        ex = eps * j0(k * r) * np.exp(-delta * k * k * t)
        return np.mean(np.abs(M1[:, 0] - ex)) / np.mean(np.abs(ex))
    g = delta * k * k / 2
    Om = np.sqrt(k * k - g * g)
    A = np.exp(-g * t) * (np.cos(Om * t) + g / Om * np.sin(Om * t))
    # A' = -k B  =>  B = -A'/k
    dA = np.exp(-g * t) * (-(Om + g * g / Om) * np.sin(Om * t))
    B = -dA / k
    exR = eps * j0(k * r) * A
    exN = eps * j1(k * r) * B
    eR = np.mean(np.abs(R1[:, 0] - exR)) / np.mean(np.abs(exR))
    eN = np.mean(np.abs(N1[:, 0] - exN)) / np.mean(np.abs(exN))
    assert np.all(M1 == 0.0)                 # no axial motion appears
    return max(eR, eN)


@pytest.mark.parametrize("which,dt", [("shear", 0.45), ("radial", 0.05), ("radial", 0.45), ("radial", 0.9)])
def test_axisymmetric_bessel_modes_converge(orc, which, dt):
    """Second order at a fixed Courant number.  The geometric terms enter as
    two half steps around the x2 sweep; that symmetric placement leaves no
    first-order splitting error, so the order holds up to CFL 0.9."""
    ns = [32, 64, 128]
    errs = [_axisym_mode_run(orc, n, which, dt) for n in ns]
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(2) for i in range(2)]
    assert errs[-1] < 1e-2, errs
    assert min(rates) > 1.6, (errs, rates)


@pytest.mark.parametrize("dt", [0.9, 0.99])
def test_axisymmetric_axis_is_stable_at_high_cfl(orc, dt):
    """Grid-scale noise on an axisymmetric grid (periodic in z, axis at y-,
    inviscid) must not grow at CFL 0.9-0.99.  Applying the geometric terms
    once after both sweeps fails this (the one-step operator of the
    first-order split scheme then has spectral radius 1.0005 at CFL 0.9 and
    the noise blows up at the axis within a few hundred steps)."""
    rng = np.random.default_rng(1)
    nx, ny, amp = 64, 24, 1e-6
    R = amp * rng.uniform(-1, 1, (ny, nx))
    M = amp * rng.uniform(-1, 1, (ny, nx))
    N = amp * rng.uniform(-1, 1, (ny, nx))
    p = orc.make_params(nx, ny, 3.5, 0.0, bc=("periodic", "periodic", "reflect", "extrap0"),
                        geometry="axisym", fixed_dt=True)
    peaks = []
    for _ in range(4):
        R, M, N, info = orc.run(p, R, M, N, 800, dt=dt)
        assert info["status"] == 0
        peaks.append(np.max(np.abs(R)))
    assert max(peaks) < 2 * amp, peaks


def test_axisymmetric_terms_are_needed(orc):
    """The same radial mode run as planar geometry misses the cylindrical terms
    and does not converge to the Bessel solution: the pin has teeth."""
    from scipy.special import j0, jn_zeros
    n, eps = 64, 1e-9
    k = jn_zeros(1, 2)[1] / n
    r = np.arange(n) + 0.5
    R0 = np.repeat((eps * j0(k * r))[:, None], 4, axis=1)
    Z = np.zeros_like(R0)
    p = orc.make_params(4, n, 3.5, 0.04, bc=("periodic", "periodic", "reflect", "reflect"),
                        geometry="planar", fixed_dt=True)
    R1, M1, N1, info = orc.run(p, R0, Z, Z, 85, dt=0.45)
    t = 85 * 0.45
    g = 0.04 * k * k / 2
    Om = np.sqrt(k * k - g * g)
    exR = eps * j0(k * r) * np.exp(-g * t) * (np.cos(Om * t) + g / Om * np.sin(Om * t))
    assert np.mean(np.abs(R1[:, 0] - exR)) / np.mean(np.abs(exR)) > 0.05


# -- Exact viscous travelling shock of the model system ------------------------

def travelling_profile(beta, delta, a, xi):
    """Exact travelling wave of the 1-D model (no tangential motion), right
    state R = -a at rest, left state R = +a.  Rankine-Hugoniot gives the speed
    V and the left momentum; the profile solves
      delta u' = -V M + u^2 + phi(R) - phi(R_R),  M = V (R - R_R),  u = M/(1+R),
    i.e. R' = H(R) (1+R)^2 / (delta V (1 + R_R)); integrated with RK4 from
    R(0) = 0 in both directions.  Returns V, R(xi), M(xi)."""
    RR, RL = -a, a
    phi = lambda R: R + (beta - 1) * R * R
    dR = RL - RR
    V = np.sqrt((phi(RL) - phi(RR)) / (dR * (1 - dR / (1 + RL) ** 2)))

    def H(R):
        M = V * (R - RR)
        u = M / (1 + R)
        return -V * M + u * u + phi(R) - phi(RR)

    def f(R):
        return H(R) * (1 + R) ** 2 / (delta * V * (1 + RR))

    xi = np.asarray(xi, dtype=float)
    out = np.empty_like(xi)
    h = 1e-3 * delta / (beta * a)
    for sign in (1, -1):
        sel = np.sign(xi) == sign if sign > 0 else xi < 0
        if sign > 0:
            sel = xi >= 0
        pts = np.sort(np.abs(xi[sel]))
        R, x, vals = 0.0, 0.0, {}
        for target in pts:
            while x < target - 1e-15:
                hh = min(h, target - x)
                s = sign * hh
                k1 = f(R); k2 = f(R + 0.5 * s * k1); k3 = f(R + 0.5 * s * k2); k4 = f(R + s * k3)
                R += s * (k1 + 2 * k2 + 2 * k3 + k4) / 6
                x += hh
            vals[target] = R
        out[sel] = [vals[abs(v)] for v in xi[sel]]
    return V, out, V * (out - RR)


@pytest.mark.slow
def test_exact_viscous_shock_profile_second_order(orc):
    beta, a = 4.0, 3e-3
    errs = []
    etas = [4, 8, 16]
    for eta in etas:
        delta = beta * a * eta            # profile width delta/(beta a) = eta cells
        nx, ny = 40 * eta, 4
        x0 = 12.0 * eta
        x = np.arange(nx) + 0.5
        V, R0, M0 = travelling_profile(beta, delta, a, x - x0)
        R0 = np.broadcast_to(R0, (ny, nx)).copy()
        M0 = np.broadcast_to(M0, (ny, nx)).copy()
        p = orc.make_params(nx, ny, beta, delta, bc=("extrap0", "extrap0", "periodic", "periodic"),
                            fixed_dt=True)
        dt = 0.5
        steps = int(round(12 * eta / dt))
        R1, M1, N1, info = orc.run(p, R0, M0, np.zeros_like(R0), steps, dt=dt)
        assert info["status"] == 0
        _, Rex, _ = travelling_profile(beta, delta, a, x - x0 - V * steps * dt)
        errs.append(np.sum(np.abs(R1[0] - Rex)) / np.sum(np.abs(Rex)))
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(2) for i in range(2)]
    assert errs[-1] < 5e-3, errs
    assert min(rates) > 1.6, (errs, rates)


def test_travelling_speed_matches_rankine_hugoniot():
    """The speed formula, checked against the closed form that the jump
    conditions give for the symmetric jump R = +-a into still medium,
    V = (1 - 2a/(1 + a)^2)^(-1/2) = 1.0029959 at a = 3e-3, and against the
    jump conditions written out independently."""
    beta, a = 4.0, 3e-3
    V, _, _ = travelling_profile(beta, 0.04, a, np.array([0.0]))
    assert abs(V - (1.0 - 2 * a / (1 + a) ** 2) ** -0.5) < 1e-12
    RL, RR = a, -a
    ML = V * (RL - RR)
    uL = ML / (1 + RL)
    flux_mom = lambda M, u, R: u * u + R + (beta - 1) * R * R
    # mass: V [R] = [M];  momentum: V [M] = [u^2 + phi]
    assert abs(V * (RL - RR) - ML) < 1e-15
    assert abs(V * ML - (flux_mom(ML, uL, RL) - flux_mom(0.0, 0.0, RR))) < 1e-15


# -- Focused source with the packet envelope (eq. hifuBC:g) -------------------

def test_packet_source_launches_the_packet_as_a_plane_wave(orc):
    """With an unfocused source covering the whole side (F -> inf, aperture
    beyond the grid) eq. hifuBC imposes q1 - 1 = q2 = g(t) at x1 = 0: a plane
    packet g = A sin(2 pi f t) exp(-(f t / W)^10) that, at small amplitude,
    propagates at c0.  The time series at a probe 80 cells in must match g
    delayed by the travel time (fitted; the face sits between 80 and 81.5
    cells away) to within 3% of A, with M = R (right-going) and N = 0.  A
    wrong envelope exponent or width, time origin, phase factor or sign of q2
    fails this."""
    eta, W, A = 40.0, 4.0, 1e-6
    f = 1.0 / eta
    p = orc.make_params(120, 4, 4.8, 0.0, bc=("source", "extrap0", "periodic", "periodic"),
                        source={"amp": A, "freq": f, "focal": 1e30, "aperture": 1e9,
                                "envelope": "packet", "packet_cycles": W})
    R = np.zeros((4, 120)); M = R.copy(); N = R.copy()
    t, dt = -6.0 / f, 0.0                 # start 6 periods before the packet centre
    ts, rs, ms, ns = [], [], [], []
    while t < 80.0 + 6.5 / f:
        R, M, N, info = orc.run(p, R, M, N, 1, t=t, dt=dt)
        assert info["status"] == 0
        t, dt = info["t"], info["dt_next"]
        ts.append(t); rs.append(R[0, 80]); ms.append(M[0, 80]); ns.append(N[0, 80])
    ts, rs, ms, ns = map(np.array, (ts, rs, ms, ns))

    def g(tt):
        return A * np.sin(2 * np.pi * f * tt) * np.exp(-(f * tt / W) ** 10)

    delays = np.linspace(79.0, 83.0, 401)
    errs = [np.max(np.abs(rs - g(ts - dly))) for dly in delays]
    k = int(np.argmin(errs))
    assert 80.0 <= delays[k] <= 81.5, delays[k]
    assert errs[k] <= 0.03 * A, errs[k] / A
    assert np.max(np.abs(ms - rs)) <= 0.03 * A
    assert np.max(np.abs(ns)) <= 1e-3 * A
    assert abs(np.max(np.abs(rs)) / A - 1.0) < 0.03      # flat top at full amplitude


def test_second_stage_turns_the_source_side_into_extrapolation(orc):
    """Sec. 4.2 runs the packet in two stages: the source on 0 <= x2 <= a and
    extrapolation beyond it, then zero-order extrapolation over the whole
    border x1 = 0.  A run that crosses the switch time must equal, bit for
    bit, a run with the source up to the first step whose t_n reaches it,
    continued from that state with an extrapolating side x- (boundary data at
    t_n).  A switch tested on t_{n+1}, a switch that keeps the source rows,
    or one that never happens fails this; so does the switch leaving the
    first stage unchanged (compared with a run with no second stage)."""
    eta, W, A = 20.0, 4.0, 2e-4
    f = 1.0 / eta
    src = {"amp": A, "freq": f, "focal": 50.0 * eta, "aperture": 10.5, "envelope": "packet",
           "packet_cycles": W}
    bc = ("source", "extrap0", "reflect", "extrap0")
    t0, dt, n1, n2 = -6.0 / f, 0.9, 120, 60
    t_switch = t0 + (n1 - 0.5) * dt          # between t_{n1-1} and t_{n1}
    mk = lambda b, stage2: orc.make_params(90, 24, 4.8, 1e-3, bc=b, fixed_dt=True,
                                           source=dict(src, stage2=stage2))
    Z = np.zeros((24, 90))
    R1, M1, N1, i1 = orc.run(mk(bc, None), Z, Z, Z, n1, t=t0, dt=dt)
    R0, M0, N0, i0 = orc.run(mk(bc, t_switch), Z, Z, Z, n1, t=t0, dt=dt)
    assert i1["status"] == 0 and i0["status"] == 0
    for a, b in ((R1, R0), (M1, M0), (N1, N0)):
        assert np.array_equal(a, b)
    assert np.max(np.abs(R1)) > 0.3 * A              # the packet has entered
    R2, M2, N2, i2 = orc.run(mk(("extrap0",) + bc[1:], None), R1, M1, N1, n2, t=i1["t"], dt=dt)
    Rs, Ms, Ns, i3 = orc.run(mk(bc, t_switch), Z, Z, Z, n1 + n2, t=t0, dt=dt)
    Rk, Mk, Nk, _ = orc.run(mk(bc, None), R1, M1, N1, n2, t=i1["t"], dt=dt)
    assert i2["status"] == 0 and i3["status"] == 0
    for a, b in ((R2, Rs), (M2, Ms), (N2, Ns)):
        assert np.array_equal(a, b)
    assert np.max(np.abs(Rk - Rs)) > 1e-3 * A         # the switch changed something


# -- Moving domain (Sec. 4: two stages, the domain follows the packet) ----------

def test_shift_moves_columns_and_fills_undisturbed_medium(orc):
    """Definition of one move of the domain by k cells along +x1."""
    rng = np.random.default_rng(11)
    R, M, N = (rng.standard_normal((3, 7)) for _ in range(3))
    for k in (0, 1, 4, 7, 9):
        R2, M2, N2 = orc.shift(R, M, N, k)
        for a, b in ((R, R2), (M, M2), (N, N2)):
            for i in range(7):
                want = a[:, i + k] if i + k < 7 else np.zeros(3)
                assert np.array_equal(b[:, i], want)


def test_moving_domain_matches_the_fixed_domain_inside_the_window(orc):
    """A focused packet (eq. hifuBC, packet envelope) run 30 periods on a
    moving domain 20 wavelengths long -- still until the packet centre
    reaches the middle of the domain at t1, then following it in jumps of 8
    cells checked every 8 steps, the source side extrapolating from t1 on --
    must equal, column for column at its current origin, the same run on a
    fixed domain 36 wavelengths long, except within 4 wavelengths of the
    trailing edge, whose extrapolated data differ from the cut-off state (the
    difference dies out within a few cells, so the rest agrees to rounding).
    A move in the wrong direction, by the wrong amount, at the wrong time or
    with anything but undisturbed medium entering on the right fails this."""
    eta, A, F, a = 8.0, 3e-4, 20.0, 4.0
    f = 1.0 / eta
    ny = int((a + 3) * eta)
    nxw, nxf = int(20 * eta), int(36 * eta)
    t0, t1 = -6.0 / f, 10.0 / f

    def params(nx):
        return orc.make_params(nx, ny, 4.8, 3e-4 * eta, bc=("source", "extrap0", "reflect", "extrap0"),
                               source={"amp": A, "freq": f, "focal": F * eta, "aperture": a * eta,
                                       "envelope": "packet", "packet_cycles": 4.0, "stage2": t1})
    steps = 266
    Rf, Mf, Nf, i_f = orc.run(params(nxf), np.zeros((ny, nxf)), np.zeros((ny, nxf)),
                              np.zeros((ny, nxf)), steps, t=t0)
    Z = np.zeros((ny, nxw))
    Rw, Mw, Nw, i_w, x_off = orc.run_window(params(nxw), Z, Z, Z, steps, t0, 0.0, t1, 8, 8)
    assert i_f["status"] == 0 and i_w["status"] == 0
    assert i_w["t"] == i_f["t"]
    assert x_off % 8 == 0 and 96 <= x_off <= i_w["t"] - t1   # moved >= 12 wavelengths, never ahead
    peak = np.max(np.abs(Rf))
    keep = slice(int(4 * eta), nxw)
    for w_, f_ in ((Rw, Rf), (Mw, Mf), (Nw, Nf)):
        ref = f_[:, x_off:x_off + nxw]
        assert np.max(np.abs(w_[:, keep] - ref[:, keep])) <= 1e-13 * peak
    assert np.max(np.abs(Rf[:, x_off:x_off + nxw])) >= 0.99 * peak   # the packet is inside


# -- Ghost rows of the intermediate state on sides with analytic data -----------

def test_analytic_y_sides_step_the_exact_plane_wave_like_periodic_rows(orc):
    """From the exact plane wave along x1 (theta_T = 0, eq. OurTaylorS,
    inviscid) at time t_n, one step with analytic data on all four sides must
    equal, bit for bit, the step with periodic rows: the state is independent
    of x2, so the x2 sweep has nothing to do.  That holds only if the ghost
    rows the x2 sweep reads went through the same x1 sweep as the interior;
    analytic Q^n written straight into them leaves an O(dt) jump at the sides
    (and the analytic state at t_n+1 an O(dt^2) one), which the x2 sweep
    turns into a change of the outer rows and a non-zero N."""
    eta, amp, nx, ny, x0 = 6.0, 1e-3, 90, 12, 30.0
    x = np.arange(nx) + 0.5
    tay = {"amp": amp, "width": eta, "x0": x0}
    pa = orc.make_params(nx, ny, 4.0, 0.0, bc=("taylor",) * 4, taylor=tay, fixed_dt=True)
    pp = orc.make_params(nx, ny, 4.0, 0.0, bc=("taylor", "taylor", "periodic", "periodic"), taylor=tay,
                         fixed_dt=True)
    for tn in (0.0, 7.25, 20.5):
        # the exact state from the oracle's own analytic data (its tanh, so the
        # interior and the ghost rows agree to the last bit)
        row = np.array([orc.taylor_value(pa, xx, 0.5, tn) for xx in x])
        R = np.broadcast_to(row[:, 0], (ny, nx)).copy()
        M = np.broadcast_to(row[:, 1], (ny, nx)).copy()
        N = np.zeros_like(R)
        Ra, Ma, Na, ia = orc.run(pa, R, M, N, 1, t=tn, dt=0.9)
        Rp, Mp, Np, ip = orc.run(pp, R, M, N, 1, t=tn, dt=0.9)
        assert ia["status"] == 0 and ip["status"] == 0
        for a, b in ((Ra, Rp), (Ma, Mp), (Na, Np)):
            assert np.array_equal(a, b)
        assert np.all(Na == 0.0) and np.max(np.abs(Ra - R)) > 1e-3 * amp


# -- Axisymmetric hoop terms: steady radial source flow --------------------------

def _steady_radial_R(beta, C, rhat):
    """R(r) of the steady inviscid radial flow N = C/r, u v r = K (r in units
    of the domain height): the radial momentum balance of the model in
    cylindrical coordinates, d(v^2 + phi(R))/dr = -v^2/r with v = C/(r(1+R)),
    phi(R) = R + (beta - 1) R^2, solved for R' and integrated with RK4 from
    R(1/2) = 0 on a fine grid."""
    def f(r, R):
        v = C / (r * (1 + R))
        return (v * v / r) / (1 + 2 * (beta - 1) * R - 2 * v * v / (1 + R))
    grid = np.linspace(0.05, 1.0, 19001)
    R = np.zeros_like(grid)
    i0 = np.searchsorted(grid, 0.5)
    for sgn in (1, -1):
        for i in (range(i0, len(grid) - 1) if sgn > 0 else range(i0, 0, -1)):
            j = i + sgn
            h, r, y = grid[j] - grid[i], grid[i], R[i]
            k1 = f(r, y)
            k2 = f(r + h / 2, y + h / 2 * k1)
            k3 = f(r + h / 2, y + h / 2 * k2)
            k4 = f(r + h, y + h * k3)
            R[j] = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return np.interp(rhat, grid, R)


def test_axisymmetric_hoop_terms_keep_a_steady_radial_flow(orc):
    """A steady, z-independent, inviscid flow in (z, r): mass gives r N = C,
    axial momentum (1/r) d(r u v)/dr = 0 gives u v r = K, radial momentum
    d(v^2 + phi)/dr + v^2/r = 0 fixes R(r) -- the balances in which the
    geometric terms -N/r, -u v/r and -v^2/r of reading R5 appear.  Started
    from this state (blended to rest near the axis, where the flow is
    singular) the scheme may move it only by its truncation error: in the band
    0.35 < r < 0.65, which neither the blend nor the outer side reaches by
    t = 0.12, the error in R, M and N converges at second order under
    refinement (64, 128, 256 rows).  A missing or sign-flipped -v^2/r or a
    missing -u v/r leaves an O(1) residual there and no convergence."""
    beta, C, K, T = 4.8, 2e-3, 1e-5, 0.12
    errs = []
    for n in (64, 128, 256):
        rj = (np.arange(n) + 0.5) / n
        R = _steady_radial_R(beta, C, rj)
        s = np.clip((rj - 0.05) / 0.1, 0.0, 1.0)
        N = C / rj * s * s * (3 - 2 * s)
        M = K * (1 + R) ** 2 / C
        Q = [np.tile(a[:, None], (1, 4)) for a in (R, M, N)]
        p = orc.make_params(4, n, beta, 0.0, bc=("periodic", "periodic", "extrap0", "extrap0"),
                            geometry="axisym")
        t, dt = 0.0, 0.0
        while t < T * n:
            R1, M1, N1, info = orc.run(p, *Q, 1, t=t, dt=dt)
            assert info["status"] == 0
            Q, t, dt = [R1, M1, N1], info["t"], info["dt_next"]
        band = (rj > 0.35) & (rj < 0.65)
        scales = (np.ptp(R[band]), np.max(np.abs(M[band])), np.max(np.abs(N[band])))
        errs.append([np.max(np.abs(q[band, 0] - e[band])) / sc for q, e, sc in zip(Q, (R, M, N), scales)])
    errs = np.array(errs)
    orders = np.log2(errs[:-1] / errs[1:])
    assert np.all(orders > 1.6), (errs, orders)
    assert errs[-1][0] < 0.05 and errs[-1][1] < 1e-5 and errs[-1][2] < 1e-4, errs


def test_focused_packet_focuses_near_f(orc):
    """The focusing delay of eq. hifuBC, tau = t + r^2/(2F): a small-amplitude
    packet from an aperture of 8 wavelengths with F = 20 wavelengths (10 cells
    per wavelength, inviscid) must peak on the axis a little before F (the
    focal shift of a finite aperture) with a gain near the 2-D estimate
    sqrt(2 a^2 / (lambda F)) = 2.5.  A delay of the wrong sign does not focus
    at all (peak at the source, gain < 1); twice the delay focuses at F/2."""
    eta, F_wl, a_wl, A = 10.0, 20.0, 8.0, 1e-6
    f = 1.0 / eta
    nx, ny = int(30 * eta), int((a_wl + 4) * eta)
    p = orc.make_params(nx, ny, 4.8, 0.0, bc=("source", "extrap0", "reflect", "extrap0"),
                        source={"amp": A, "freq": f, "focal": F_wl * eta, "aperture": a_wl * eta,
                                "envelope": "packet", "packet_cycles": 4.0})
    Q = [np.zeros((ny, nx)) for _ in range(3)]
    t, dt = -6.0 / f, 0.0
    pmax = np.zeros(nx)
    while t < (30 + 6.5) / f:
        R, M, N, info = orc.run(p, *Q, 1, t=t, dt=dt)
        assert info["status"] == 0
        Q, t, dt = [R, M, N], info["t"], info["dt_next"]
        np.maximum(pmax, R[0], out=pmax)
    k = int(np.argmax(pmax))
    x_over_f, gain = (k + 0.5) / eta / F_wl, pmax[k] / A
    assert 0.75 < x_over_f < 0.98, x_over_f
    assert 1.8 < gain < 2.6, gain


# ---------------------------------------------------------------------------
# CFL control: rejection and redo (opening of Sec. 4; reading R4).  A step whose
# CFL number exceeds nu_max is discarded and redone from the same Q^n with
# dt nu_W / nu.  Pinned against single attempts at the two time steps: the
# rejected-then-redone run must equal, bit for bit, one fresh attempt at the
# redone step from Q^n.
# ---------------------------------------------------------------------------

def _redo_case(orc):
    from common import dimless_state, oracle_params, pulse_workload
    w = pulse_workload(40, 32, ("extrap0", "extrap0", "reflect", "extrap0"), seed=11)
    p = oracle_params(orc, w)
    pf = oracle_params(orc, w, fixed_dt=True)
    R, M, N = dimless_state(w)
    return p, pf, R, M, N


def test_rejected_step_is_redone_from_the_same_state(orc):
    p, pf, R, M, N = _redo_case(orc)
    assert p.cfl_max == 1.0 and p.cfl_target == 0.9
    dt_bad = 3.0 * p.cfl_target / orc.dry_smax(p, R, M, N)
    # the first attempt on its own (fixed dt: nu recorded, never rejected)
    _, _, _, a1 = orc.run(pf, R, M, N, 1, dt=dt_bad)
    nu1 = a1["nu_last"]
    assert nu1 > p.cfl_max
    dt_redo = dt_bad * p.cfl_target / nu1
    # the adaptive run from dt_bad: one rejection, then the redo
    Ra, Ma, Na, ia = orc.run(p, R, M, N, 1, dt=dt_bad)
    assert ia["status"] == orc.OK and ia["rejected"] == 1 and ia["steps"] == 1
    # one fresh attempt at dt_redo from the same Q^n
    Rb, Mb, Nb, ib = orc.run(pf, R, M, N, 1, dt=dt_redo)
    assert ib["nu_last"] <= p.cfl_max
    for x, y in zip((Ra, Ma, Na), (Rb, Mb, Nb)):
        assert np.array_equal(x, y)
    assert ia["t"] == dt_redo
    assert ia["nu_last"] == ib["nu_last"]
    assert ia["dt_next"] == dt_redo * p.cfl_target / ib["nu_last"]
    # the input is not the answer: the redone step did change the state
    assert not np.array_equal(Ra, R)


def test_no_retries_left_keeps_the_state(orc):
    p, pf, R, M, N = _redo_case(orc)
    p.max_retries = 0
    dt_bad = 3.0 * p.cfl_target / orc.dry_smax(p, R, M, N)
    R1, M1, N1, info = orc.run(p, R, M, N, 3, dt=dt_bad)
    assert info["status"] == orc.E_RETRIES
    assert info["steps"] == 0 and info["rejected"] == 1 and info["status_step"] == 0
    for x, y in zip((R1, M1, N1), (R, M, N)):
        assert np.array_equal(x, y)
    # with one retry allowed the same run succeeds
    p.max_retries = 1
    _, _, _, info = orc.run(p, R, M, N, 3, dt=dt_bad)
    assert info["status"] == orc.OK and info["steps"] == 3 and info["rejected"] == 1


def test_moving_domain_with_taylor_sides_matches_the_fixed_domain(orc):
    """An oblique Taylor shock (theta_T = pi/8, eq. OurTaylorS rotated) with
    analytic data on all four sides, run on a domain 96 cells wide that stays
    still until the front's trace on the middle row reaches the middle column
    at t1 and then follows it along x1 at the trace speed 1/cos(theta_T) in
    jumps of 4 cells, must equal, column for column at its current origin, the
    same run on a fixed domain 200 cells wide with the same rows, except
    within 20 cells of the trailing edge: there the fixed run holds the waves
    the front sheds backwards, which the moving domain's analytic side cuts
    off (the difference dies out within 17 cells).  The data on every side are
    taken at path coordinates and the entering columns hold the profile (the
    medium ahead of the front, uniform to the last bit on both runs).  A move
    in the wrong direction, by the wrong amount, or data anchored on the domain
    instead of the path fails this."""
    th = math.pi / 8
    c, s = math.cos(th), math.sin(th)
    amp, width, beta = 1e-3, 1.5, 3.5
    delta = beta * amp * width              # travelling-wave balance of eq. OurTaylorS
    ny, nxw, nxf = 24, 96, 200
    xmid = nxw / 2
    x0 = 24.0                                # front through (x0, 0) at t = 0 (xi = 0)
    tay = {"amp": amp, "width": width, "x0": x0, "y0": 0.0, "angle": th}

    def params(nx):
        return orc.make_params(nx, ny, beta, delta, bc=("taylor",) * 4, taylor=tay)

    def state(p, nx):
        q = np.array([[orc.taylor_value(p, i + 0.5, j + 0.5, 0.0) for i in range(nx)] for j in range(ny)])
        return q[..., 0], q[..., 1], q[..., 2]

    pf, pw = params(nxf), params(nxw)
    # trace of the front on the middle row: xi = 0 at x = x0 - y s / c + t / c
    t1 = (xmid - (x0 - (ny / 2) * s / c)) * c
    steps = 90
    Rf, Mf, Nf, i_f = orc.run(pf, *state(pf, nxf), steps)
    Rw, Mw, Nw, i_w, x_off = orc.run_window(pw, *state(pw, nxw), steps, 0.0, 0.0, t1, 5, 4, speed=1.0 / c)
    assert i_f["status"] == 0 and i_w["status"] == 0
    assert i_w["t"] == i_f["t"] and t1 > 5.0 and i_w["t"] > t1 + 40.0
    assert x_off == 4 * math.floor((i_w["t"] - t1) / c / 4) and x_off >= 40
    keep = slice(20, nxw)
    for w_, f_ in ((Rw, Rf), (Mw, Mf), (Nw, Nf)):
        assert np.max(np.abs(w_[:, keep] - f_[:, x_off:x_off + nxw][:, keep])) <= 1e-13 * amp
    # the front crosses the middle row inside the compared columns, and the
    # trailing edge does differ (the comparison is not vacuous there)
    row = Rw[ny // 2]
    k = int(np.argmin(np.abs(row)))
    assert 30 <= k <= nxw - 20 and abs(row[k]) < 0.3 * amp and row[-1] == -amp
    assert np.max(np.abs(Rw[:, :4] - Rf[:, x_off:x_off + 4])) > 1e-8 * amp
    # columns entering right after a move hold the profile at their path
    # coordinates and the time of the move (here near the front, where the
    # profile is not uniform): one chunk of 5 steps, then the move
    tay["x0"] = 34.0                          # the front close to the right side
    pn, pp = params(40), params(nxf)
    Rn, Mn, Nn, i_n, xo = orc.run_window(pn, *state(pn, 40), 5, 0.0, 0.0, 0.0, 5, 4, speed=2.7)
    assert i_n["status"] == 0 and xo == 4 * math.floor(i_n["t"] * 2.7 / 4) and 8 <= xo < 40
    for i in range(40 - xo, 40):
        for j in range(ny):
            want = orc.taylor_value(pp, xo + i + 0.5, j + 0.5, i_n["t"])
            got = np.array([Rn[j, i], Mn[j, i], Nn[j, i]])
            assert np.max(np.abs(got - want)) <= 1e-15 * amp
    assert np.min(np.abs(Rn[:, 40 - xo:])) < 0.9 * amp
