"""Pins for the oracle's Runge-Kutta drivers (section "FR Algorithm": explicit RK in time).

The same driver that advances the FR residual is applied to scalar ODEs with exact solutions;
both schemes must show fourth-order convergence, which fails for any mistyped coefficient.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("scheme", ["rk4", "lsrk45"])
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
