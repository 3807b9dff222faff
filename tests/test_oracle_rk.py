"""Pins for the five-stage low-storage Runge-Kutta scheme (oracle).

Exact rational arithmetic on the test equation y' = z y gives the stability
polynomial, whose first five coefficients must be those of exp(z) (fourth
order); the stage times c_i must equal the time reached by the stages on
y' = 1; and the global error on y' = cos t must fall 16-fold per halving.
"""
from fractions import Fraction

import numpy as np

from oracle.timestep import RK4A, RK4B, RK4C, lserk_step


def _polymul_z(p):
    return [Fraction(0)] + p


def _axpy(a, x, y):
    n = max(len(x), len(y))
    x = x + [Fraction(0)] * (n - len(x))
    y = y + [Fraction(0)] * (n - len(y))
    return [a * xi + yi for xi, yi in zip(x, y)]


def test_stability_polynomial():
    y = [Fraction(1)]
    res = [Fraction(0)]
    for a, b in zip(RK4A, RK4B):
        res = _axpy(a, res, _polymul_z(y))     # res = a res + z y
        y = _axpy(b, res, y)                   # y = y + b res
    expect = [Fraction(1), Fraction(1), Fraction(1, 2), Fraction(1, 6), Fraction(1, 24)]
    # the published 13-digit rationals meet the order conditions to ~1e-25
    assert all(abs(float(c - e)) < 1e-20 for c, e in zip(y[:5], expect))
    assert abs(float(y[5]) - 1 / 200) < 1e-12
    assert len(y) == 6


def test_stage_times():
    # y' = 1, y(0) = 0: after stage i the state equals c_{i+1} (dt = 1)
    y, res = Fraction(0), Fraction(0)
    for i in range(5):
        res = RK4A[i] * res + 1
        y = y + RK4B[i] * res
        if i < 4:
            assert abs(float(y - RK4C[i + 1])) < 1e-12
    assert abs(float(y) - 1.0) < 1e-14


def test_fourth_order_convergence():
    def f(y, t):
        return np.cos(t) * np.ones_like(y)

    errs = []
    for n in (10, 20, 40):
        dt = 2.0 / n
        y = np.zeros(1)
        for k in range(n):
            y, _ = lserk_step(f, y, k * dt, dt)
        errs.append(abs(y[0] - np.sin(2.0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8), rates
