"""Pins of the oracle's ghost cells: every side rule, cell by cell, on both
ghost layers (CPU).

What fixes each rule:
  * focused source (Sec. 4.2, eq. hifuBC): the density perturbation is g(r, t)
    and the momentum has magnitude |g| along the line from the source point
    (0, r) to the focus (F, 0) -- towards the focus where g > 0 -- so that
    the ghost momentum (q^2, q^3) = g (F, -r)/h, h = sqrt(r^2 + F^2);
    outside the aperture, and everywhere on the side once the second stage
    has started, the side is zero-order extrapolation (Sec. 4.2 border rules);
  * Taylor (Sec. 4.1, eq. OurTaylorS rotated by theta_T): the right-going
    simple wave, momentum = R times the unit propagation vector;
  * reflection: mirror image with the normal momentum negated;
  * zero-order extrapolation and periodic wrap: copies of interior cells.
"""
import math

import numpy as np
import pytest

NX, NY = 12, 10


def _state(seed):
    rng = np.random.default_rng(seed)
    R = 1e-3 * rng.uniform(-1, 1, (NY, NX))
    M = 1e-3 * rng.uniform(-1, 1, (NY, NX))
    N = 1e-3 * rng.uniform(-1, 1, (NY, NX))
    return R, M, N


def _frame(side, layer):
    """Ghost cells of one side and layer: list of (gi, gj)."""
    if side == 0:
        return [(-layer, j) for j in range(NY)]
    if side == 1:
        return [(NX - 1 + layer, j) for j in range(NY)]
    if side == 2:
        return [(i, -layer) for i in range(NX)]
    return [(i, NY - 1 + layer) for i in range(NX)]


def _source_params(orc, envelope="ramp", stage2=None, aperture=6.0):
    src = {"amp": 2e-4, "freq": 0.05, "focal": 25.0, "aperture": aperture, "ramp_cycles": 3.0,
           "envelope": envelope, "packet_cycles": 4.0, "stage2": stage2}
    return orc.make_params(NX, NY, 3.5, 0.01, bc=("source", "extrap0", "reflect", "extrap0"),
                           source=src), src


def _g(src, r, t):
    """eq. hifuBC: amplitude x envelope x sin(2 pi f tau), tau = t + r^2/(2F)."""
    f, F = src["freq"], src["focal"]
    tau = t + r * r / (2.0 * F)
    if src["envelope"] == "packet":
        env = math.exp(-((f * tau / src["packet_cycles"]) ** 10))
    else:
        tr = src["ramp_cycles"] / f
        env = 0.0 if t <= 0 else (math.sin(math.pi * f * t / (2 * src["ramp_cycles"])) ** 2 if t < tr else 1.0)
    return src["amp"] * env * math.sin(2 * math.pi * f * tau)


@pytest.mark.parametrize("t", [61.0, 73.3, 88.8])
def test_source_ghost_momentum_points_at_the_focus(orc, t):
    p, src = _source_params(orc)
    R, M, N = _state(1)
    F = src["focal"]
    inside = 0
    for layer in (1, 2):
        for gi, gj in _frame(0, layer):
            q = orc.ghost(p, R, M, N, t, 0, gi, gj, layer)
            r = gj + 0.5
            if r > src["aperture"]:
                # outside the aperture: zero-order extrapolation of the row
                assert np.array_equal(q, [R[gj, 0], M[gj, 0], N[gj, 0]])
                continue
            inside += 1
            g = _g(src, r, t)
            assert abs(q[0] - g) <= 1e-15 * src["amp"]
            h = math.hypot(r, F)
            ex, ey = F / h, -r / h               # unit vector from (0, r) towards the focus (F, 0)
            along = q[1] * ex + q[2] * ey
            across = -q[1] * ey + q[2] * ex
            assert abs(along - g) <= 2e-15 * src["amp"], (gj, along, g)
            assert abs(across) <= 2e-15 * src["amp"], (gj, across)
            # towards the focus where g > 0: into the domain and towards the symmetry line
            if abs(g) > 1e-3 * src["amp"]:
                assert np.sign(q[1]) == np.sign(g) and np.sign(q[2]) == -np.sign(g)
    assert inside == 2 * 6


def test_source_ghost_layers_are_equal_and_envelopes(orc):
    R, M, N = _state(2)
    for env, times in (("ramp", [0.0, 5.0, 30.0, 59.9]), ("packet", [-120.0, -40.0, 0.0, 35.0])):
        p, src = _source_params(orc, envelope=env)
        for t in times:
            for j in range(6):
                q1 = orc.ghost(p, R, M, N, t, 0, -1, j, 1)
                q2 = orc.ghost(p, R, M, N, t, 0, -2, j, 2)
                assert np.array_equal(q1, q2)
                g = _g(src, j + 0.5, t)
                assert abs(q1[0] - g) <= 1e-15 * src["amp"], (env, t, j, q1[0], g)
    # before the ramp starts the source is at rest
    p, src = _source_params(orc)
    assert np.array_equal(orc.ghost(p, R, M, N, 0.0, 0, -1, 0, 1), [0.0, 0.0, 0.0])


def test_source_side_is_extrapolation_in_the_second_stage(orc):
    R, M, N = _state(3)
    p, src = _source_params(orc, stage2=70.0)
    for t, second in ((69.99, False), (70.0, True), (95.0, True)):
        for layer in (1, 2):
            for gi, gj in _frame(0, layer):
                q = orc.ghost(p, R, M, N, t, 0, gi, gj, layer)
                copy = [R[gj, 0], M[gj, 0], N[gj, 0]]
                if second or gj + 0.5 > src["aperture"]:
                    assert np.array_equal(q, copy)
                else:
                    assert abs(q[0] - _g(src, gj + 0.5, t)) <= 1e-15 * src["amp"]


@pytest.mark.parametrize("angle", [0.0, math.pi / 16, math.pi / 4, 2.0])
def test_taylor_ghost_is_the_rotated_simple_wave(orc, angle):
    amp, width, x0, y0 = 3e-4, 1.7, 4.0, 2.0
    p = orc.make_params(NX, NY, 3.5, 0.01, bc=("taylor",) * 4,
                        taylor={"amp": amp, "width": width, "x0": x0, "y0": y0, "angle": angle})
    R, M, N = _state(4)
    ca, sa = math.cos(angle), math.sin(angle)
    for t in (0.0, 2.5, 6.0):
        for side in range(4):
            for layer in (1, 2):
                for gi, gj in _frame(side, layer):
                    q = orc.ghost(p, R, M, N, t, side, gi, gj, layer)
                    x, y = gi + 0.5, gj + 0.5                     # the ghost cell's centre
                    xi = (x - x0) * ca + (y - y0) * sa
                    Rx = -amp * math.tanh((xi - t) / width)
                    assert abs(q[0] - Rx) <= 2e-16 * amp
                    # simple wave: momentum along the propagation direction, equal to R
                    assert abs(q[1] * ca + q[2] * sa - q[0]) <= 4e-16 * amp
                    assert abs(-q[1] * sa + q[2] * ca) <= 4e-16 * amp


def _rule_ghost(R, M, N, side, gi, gj, layer, rule):
    """The expected ghost by the plain statement of each rule."""
    if side == 0:
        src = {"periodic": (NX - layer, gj), "extrap0": (0, gj), "reflect": (layer - 1, gj)}[rule]
    elif side == 1:
        src = {"periodic": (layer - 1, gj), "extrap0": (NX - 1, gj), "reflect": (NX - layer, gj)}[rule]
    elif side == 2:
        src = {"periodic": (gi, NY - layer), "extrap0": (gi, 0), "reflect": (gi, layer - 1)}[rule]
    else:
        src = {"periodic": (gi, layer - 1), "extrap0": (gi, NY - 1), "reflect": (gi, NY - layer)}[rule]
    i, j = src
    q = np.array([R[j, i], M[j, i], N[j, i]])
    if rule == "reflect":
        q[1 if side < 2 else 2] *= -1.0
    return q


@pytest.mark.parametrize("rule", ["periodic", "extrap0", "reflect"])
def test_state_rules_copy_the_right_interior_cells(orc, rule):
    p = orc.make_params(NX, NY, 3.5, 0.01, bc=(rule,) * 4)
    R, M, N = _state(5)
    for side in range(4):
        for layer in (1, 2):
            for gi, gj in _frame(side, layer):
                q = orc.ghost(p, R, M, N, 1.0, side, gi, gj, layer)
                assert np.array_equal(q, _rule_ghost(R, M, N, side, gi, gj, layer, rule)), (side, gi, gj)


def test_reflection_makes_the_wall_a_mirror(orc):
    """Geometric statement of reflection: the state with its ghosts is symmetric
    about the wall, with the normal momentum odd and the rest even."""
    p = orc.make_params(NX, NY, 3.5, 0.01, bc=("reflect",) * 4)
    R, M, N = _state(6)
    for layer in (1, 2):
        for j in range(NY):
            g = orc.ghost(p, R, M, N, 0.0, 0, -layer, j, layer)     # x = -layer + 1/2
            m = (R[j, layer - 1], M[j, layer - 1], N[j, layer - 1])  # x = +layer - 1/2
            assert (g[0], g[1], g[2]) == (m[0], -m[1], m[2])
        for i in range(NX):
            g = orc.ghost(p, R, M, N, 0.0, 3, i, NY - 1 + layer, layer)
            m = (R[NY - layer, i], M[NY - layer, i], N[NY - layer, i])
            assert (g[0], g[1], g[2]) == (m[0], m[1], -m[2])


def test_ghost_rejects_cells_off_the_frame(orc):
    p = orc.make_params(NX, NY, 3.5, 0.01)
    R, M, N = _state(7)
    for side, gi, gj, layer in ((0, -1, NY, 1), (0, 0, 0, 1), (1, NX, 0, 2), (2, 0, -3, 3), (3, NX, NY, 1)):
        with pytest.raises(ValueError):
            orc.ghost(p, R, M, N, 0.0, side, gi, gj, layer)
