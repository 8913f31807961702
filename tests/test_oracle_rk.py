"""Pins for the oracle's Runge-Kutta drivers (section "FR Algorithm": explicit RK in time).

The same driver that advances the FR residual is applied to scalar ODEs with exact solutions;
both schemes must show fourth-order convergence, which fails for any mistyped coefficient.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("scheme", ["rk4", "lsrk45", "ssprk104"])
@pytest.mark.parametrize("ode", [0, 1])
def test_fourth_order(scheme, ode):
    T = 1.0
    errs = []
    for n in (10, 20, 40):
        dt = T / n
        y = oracle.rk_scalar(scheme, ode, -1.3, 1.0, dt, n)
        exact = np.exp(-1.3 * T) if ode == 0 else 1.0 / (1.0 + T)
        errs.append(abs(y[-1] - exact))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.7), (errs, rates)
    assert np.all(rates < 4.6), (errs, rates)


def test_rk4_real_axis_stability_limit():
    # classical RK4's stability polynomial 1 + z + z^2/2 + z^3/6 + z^4/24 has |R(z)| = 1 at
    # z ~ -2.785 on the negative real axis
    assert abs(oracle.rk_scalar("rk4", 0, -2.7, 1.0, 1.0, 200)[-1]) < 1.0
    assert abs(oracle.rk_scalar("rk4", 0, -2.9, 1.0, 1.0, 200)[-1]) > 1.0


def test_lsrk45_real_axis_stability_limit():
    # the fifth stage buys the Carpenter-Kennedy scheme a real-axis stability interval well
    # beyond RK4's (|z| ~ 2.785): it is stable at z = -4.2, where RK4 diverges
    assert abs(oracle.rk_scalar("lsrk45", 0, -4.2, 1.0, 1.0, 200)[-1]) < 1.0
    assert abs(oracle.rk_scalar("rk4", 0, -4.2, 1.0, 1.0, 20)[-1]) > 1.0


def _stability_polynomial(scheme, degree):
    """Coefficients of R(z) (y1 = R(z) y0 for y' = lambda y, z = lambda dt), recovered from the
    oracle's one-step map at Chebyshev points by polynomial interpolation."""
    z = -1.0 + np.cos(np.pi * (np.arange(degree + 1) + 0.5) / (degree + 1))  # in [-2, 0]
    y = np.array([oracle.rk_scalar(scheme, 0, zi, 1.0, 1.0, 1)[-1] for zi in z])
    return np.polynomial.polynomial.polyfit(z, y, degree)


def test_ssprk104_stability_polynomial_order():
    """Ketcheson's SSPRK(10,4): R(z) matches exp(z) through z^4 and has degree 10."""
    import math

    c = _stability_polynomial("ssprk104", 10)
    for k in range(5):
        assert abs(c[k] - 1.0 / math.factorial(k)) < 1e-9, (k, c[k])
    assert abs(c[5] - 1.0 / 120) > 1e-4  # not exp(z) beyond fourth order


def test_ssprk104_preserves_monotonicity_to_six_euler_steps():
    """Upwind advection is monotone under forward Euler for dt <= 1. A strong-stability-
    preserving method with SSP coefficient 6 keeps a step profile within [0, 1] for every
    dt <= 6; classical RK4 (coefficient < 1 for this problem) does not at dt = 1.5."""
    u0 = np.zeros(64)
    u0[10:30] = 1.0
    for dt in (1.0, 3.0, 6.0):
        u = oracle.rk_upwind("ssprk104", u0, dt, 40)
        assert u.min() >= -1e-13 and u.max() <= 1 + 1e-13, (dt, u.min(), u.max())
    u = oracle.rk_upwind("rk4", u0, 1.5, 40)
    assert u.min() < -1e-6 or u.max() > 1 + 1e-6
    # beyond the SSP coefficient monotonicity is lost
    u = oracle.rk_upwind("ssprk104", u0, 7.5, 40)
    assert u.min() < -1e-6 or u.max() > 1 + 1e-6


def test_ssprk104_real_axis_stability():
    # ten stages of dt/6: stable much further along the negative real axis than RK4
    assert abs(oracle.rk_scalar("ssprk104", 0, -12.0, 1.0, 1.0, 200)[-1]) < 1.0
    assert abs(oracle.rk_scalar("ssprk104", 0, -16.0, 1.0, 1.0, 50)[-1]) > 1.0
