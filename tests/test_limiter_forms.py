"""The limited wave strengths the step kernel forms without dividing by alpha
(Sec. 3.1, MC limiter), checked in FP64 on the host against the textbook
form alpha * psi(theta), psi = phi / 2, phi(theta) = max(0, min((1 + theta)/2,
2, 2 theta)), theta = t / (alpha n):

* the sign form of the FP64 kernel: with u = t / n and g the sign of alpha,
  psi alpha = g max(0, min((|alpha| + g u)/4, |alpha|, g u));
* the median form of the FP32 kernel's shear family (n = 1): with
  q = (alpha + t)/4, psi alpha = med3(0, min(q, alpha, t), max(q, alpha, t)).

Both are exact algebra (they differ from the textbook form by rounding
only), and both give 0 for alpha = 0, where the textbook form needs the
guard theta := 0.  A planted mistake (a dropped /4, a sign left off u, a
missing clamp) fails these checks."""
import numpy as np

import pytest


def _textbook(a, t, n):
    with np.errstate(divide="ignore", invalid="ignore"):
        th = np.where(a != 0.0, t / (a * n), 0.0)
    phi = np.maximum(0.0, np.minimum(np.minimum((1.0 + th) / 2.0, 2.0), 2.0 * th))
    return a * phi / 2.0


def _sign_form(a, t, n):
    u = t / n
    g = np.where(np.signbit(a), -1.0, 1.0)
    aa = np.abs(a)
    m = np.maximum(0.0, np.minimum(np.minimum((aa + g * u) / 4.0, aa), g * u))
    return g * m


def _median_form(a, t):
    q = (a + t) / 4.0
    lo = np.minimum(np.minimum(q, a), t)
    hi = np.maximum(np.maximum(q, a), t)
    return np.median(np.stack([np.zeros_like(a), lo, hi]), axis=0)


def _samples(seed):
    rng = np.random.default_rng(seed)
    k = 200_000
    a = rng.standard_normal(k) * 10.0 ** rng.uniform(-6, 2, k)
    t = rng.standard_normal(k) * 10.0 ** rng.uniform(-6, 2, k)
    # every regime: equal and opposite signs, theta near 0, 1/3, 1, 3 and large
    c = rng.choice([0.0, 1.0 / 3.0, 1.0, 3.0, -1.0, 1e-9], size=k)
    pick = rng.random(k) < 0.3
    t = np.where(pick, a * c * (1.0 + 1e-12 * rng.standard_normal(k)), t)
    a[:50] = 0.0
    t[50:100] = 0.0
    return a, t


@pytest.mark.parametrize("seed", [1, 2])
def test_sign_form_equals_the_textbook_limiter(seed):
    a, t = _samples(seed)
    n = 1.0 + np.random.default_rng(seed + 10).uniform(0.0, 5.0, a.shape)
    ref = _textbook(a, t, n)
    got = _sign_form(a, t, n)
    scale = np.maximum(np.abs(a), np.abs(t / n))
    assert np.all(np.abs(got - ref) <= 4e-16 * scale + 1e-300)
    assert np.all(got[:50] == 0.0)


@pytest.mark.parametrize("seed", [3, 4])
def test_median_form_equals_the_textbook_limiter_for_unit_eigenvectors(seed):
    a, t = _samples(seed)
    ref = _textbook(a, t, 1.0)
    got = _median_form(a, t)
    scale = np.maximum(np.abs(a), np.abs(t))
    assert np.all(np.abs(got - ref) <= 4e-16 * scale + 1e-300)
    assert np.all(got[:50] == 0.0)


def test_the_checks_see_a_planted_mistake():
    a, t = _samples(5)
    ref = _textbook(a, t, 1.0)
    scale = np.maximum(np.abs(a), np.abs(t))

    def no_quarter(a, t):               # (alpha + t) without the 1/4
        lo = np.minimum(np.minimum(a + t, a), t)
        hi = np.maximum(np.maximum(a + t, a), t)
        return np.median(np.stack([np.zeros_like(a), lo, hi]), axis=0)

    def no_clamp(a, t):                 # the minimum alone, no median with 0
        return np.minimum(np.minimum((a + t) / 4.0, a), t)

    def unsigned_u(a, t):               # the sign form without g on u
        aa = np.abs(a)
        g = np.where(np.signbit(a), -1.0, 1.0)
        return g * np.maximum(0.0, np.minimum(np.minimum((aa + t) / 4.0, aa), t))

    for bad in (no_quarter, no_clamp, unsigned_u):
        assert np.any(np.abs(bad(a, t) - ref) > 1e-3 * scale), bad.__name__
