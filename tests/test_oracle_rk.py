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


# Carpenter and Kennedy's published stage nodes c_i of the five-stage scheme, a separate set of
# ratios from the 2N coefficients. They are rounded independently: the row sums of the tableau
# reproduce them to 8e-12, except c_2 (3.8e-8).
LSRK45_C = ["0", "1432997174477/9575080441237", "2526269341429/6820363266787",
            "2006345519317/3224310063776", "2802321613138/2924317926251"]


def _butcher_from_2n(A, B):
    """Butcher tableau (a, b, c) of the 2N scheme dU <- A_i dU + dt R(U); U <- U + B_i dU, in
    exact rational arithmetic on the given binary values. Stage i is evaluated at
    U_0 + sum_j a_ij k_j with k_j = dt R of stage j; the register after stage l holds
    sum_{j <= l} (prod_{m = j+1..l} A_m) k_j."""
    from fractions import Fraction

    A = [Fraction(x) for x in A]
    B = [Fraction(x) for x in B]
    s = len(A)

    def weight(i_last, j):  # coefficient of k_j in U after stage i_last
        tot = Fraction(0)
        for l in range(j, i_last + 1):
            prod = Fraction(1)
            for m in range(j + 1, l + 1):
                prod *= A[m]
            tot += B[l] * prod
        return tot

    a = [[weight(i - 1, j) if j < i else Fraction(0) for j in range(s)] for i in range(s)]
    b = [weight(s - 1, j) for j in range(s)]
    c = [sum(row) for row in a]
    return a, b, c


def test_lsrk45_tables_satisfy_the_fourth_order_conditions():
    """The eight order conditions of a fourth-order Runge-Kutta method (the rooted trees of
    order <= 4), evaluated exactly on the oracle's double-precision 2N coefficients, and the
    Butcher row sums against the published nodes c_i."""
    from fractions import Fraction

    A, B = oracle.lsrk45_tables()
    a, b, c = _butcher_from_2n(A, B)
    s = len(b)
    ac = [sum(a[i][j] * c[j] for j in range(s)) for i in range(s)]
    ac2 = [sum(a[i][j] * c[j] ** 2 for j in range(s)) for i in range(s)]
    aac = [sum(a[i][j] * ac[j] for j in range(s)) for i in range(s)]
    conds = {
        "sum b = 1": (sum(b), Fraction(1)),
        "b.c = 1/2": (sum(b[i] * c[i] for i in range(s)), Fraction(1, 2)),
        "b.c^2 = 1/3": (sum(b[i] * c[i] ** 2 for i in range(s)), Fraction(1, 3)),
        "b.Ac = 1/6": (sum(b[i] * ac[i] for i in range(s)), Fraction(1, 6)),
        "b.c^3 = 1/4": (sum(b[i] * c[i] ** 3 for i in range(s)), Fraction(1, 4)),
        "b.(c*Ac) = 1/8": (sum(b[i] * c[i] * ac[i] for i in range(s)), Fraction(1, 8)),
        "b.Ac^2 = 1/12": (sum(b[i] * ac2[i] for i in range(s)), Fraction(1, 12)),
        "b.AAc = 1/24": (sum(b[i] * aac[i] for i in range(s)), Fraction(1, 24)),
    }
    for name, (got, want) in conds.items():
        assert abs(float(got - want)) <= 1e-11, (name, float(got - want))
    # not fifth order: the scheme's order is exactly four
    assert abs(float(sum(b[i] * c[i] ** 4 for i in range(s)) - Fraction(1, 5))) > 1e-6
    for i in range(s):
        assert abs(float(c[i] - Fraction(LSRK45_C[i]))) <= (5e-8 if i == 2 else 1e-11), (i, float(c[i]))


def test_lsrk45_tables_catch_a_perturbed_digit():
    """Negative control: one coefficient off in its twelfth significant digit breaks an order
    condition by more than the 1e-11 tolerance."""
    from fractions import Fraction

    A, B = oracle.lsrk45_tables()
    B = B.copy()
    B[2] *= 1 + 1e-10
    a, b, c = _butcher_from_2n(A, B)
    assert abs(float(sum(b) - 1)) > 1e-11


def test_lsrk45_driver_uses_its_tables():
    """The stability polynomial the driver realises equals the one of the tableau: coefficients
    1, 1, 1/2, 1/6, 1/24 (fourth order) and b A^3 c for z^5."""
    import math

    A, B = oracle.lsrk45_tables()
    a, b, c = _butcher_from_2n(A, B)
    s = len(b)
    Ac = [sum(a[i][j] * c[j] for j in range(s)) for i in range(s)]
    AAc = [sum(a[i][j] * Ac[j] for j in range(s)) for i in range(s)]
    AAAc = [sum(a[i][j] * AAc[j] for j in range(s)) for i in range(s)]
    c5 = float(sum(b[i] * AAAc[i] for i in range(s)))
    coef = _stability_polynomial("lsrk45", 5)
    for k in range(5):
        assert abs(coef[k] - 1.0 / math.factorial(k)) < 1e-9, (k, coef[k])
    assert abs(coef[5] - c5) < 1e-9, (coef[5], c5)
