"""Pins for the oracle's physical and numerical fluxes (Eq. (1); interface Riemann solvers).

Each pin is a property or a special case with a closed form, not a re-typed formula:
* consistency F*(U, U, n) = F(U).n and conservation F*(L, R, n) = -F*(R, L, -n);
* rotational invariance of the inviscid and viscous fluxes;
* Roe: fully supersonic states give pure upwinding; a stationary contact is resolved exactly;
* Rusanov: at a stationary contact the only dissipation is -(1/2) max(c_L, c_R) * jump(rho);
* viscous flux: simple shear, pure dilatation and pure conduction have textbook stresses.
"""
import math

import numpy as np
import pytest

import oracle

G = 1.4
rng = np.random.default_rng(0)


def cons(rho, u, p):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * u @ u])


def random_state(r):
    return cons(r.uniform(0.5, 2.0), r.normal(size=3) * 0.6, r.uniform(0.5, 3.0))


def unit(r):
    n = r.normal(size=3)
    return n / np.linalg.norm(n)


def rotation(r):
    q, _ = np.linalg.qr(r.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def rot_state(Q, U):
    V = U.copy()
    V[1:4] = Q @ U[1:4]
    return V


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_consistency_and_conservation(flux):
    r = np.random.default_rng(1)
    for _ in range(50):
        UL, UR, n = random_state(r), random_state(r), unit(r)
        F = oracle.riemann(flux, UL, UL, n)
        assert np.allclose(F, oracle.inviscid_flux(UL, n), rtol=1e-13, atol=1e-13)
        a = oracle.riemann(flux, UL, UR, n)
        b = oracle.riemann(flux, UR, UL, -n)
        assert np.allclose(a, -b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_rotational_invariance(flux):
    r = np.random.default_rng(2)
    for _ in range(20):
        UL, UR, n, Q = random_state(r), random_state(r), unit(r), rotation(r)
        F = oracle.riemann(flux, UL, UR, n)
        Fr = oracle.riemann(flux, rot_state(Q, UL), rot_state(Q, UR), Q @ n)
        assert np.allclose(Fr, rot_state(Q, F), rtol=1e-12, atol=1e-12)


def test_inviscid_flux_at_rest_is_pressure():
    n = unit(rng)
    U = cons(1.3, [0, 0, 0], 2.1)
    F = oracle.inviscid_flux(U, n)
    assert np.allclose(F, [0, *(2.1 * n), 0], atol=1e-15)


def test_roe_supersonic_is_upwind():
    r = np.random.default_rng(3)
    for _ in range(20):
        n = unit(r)
        c = 1.0
        # both states move along +n at Mach >= 3 (rho = 1.4 p keeps c = 1)
        UL = cons(1.0, 3.5 * n + 0.1 * r.normal(size=3), 1.0 / 1.4)
        UR = cons(1.1, 3.2 * n + 0.1 * r.normal(size=3), 1.1 / 1.4)
        F = oracle.riemann("roe", UL, UR, n)
        assert np.allclose(F, oracle.inviscid_flux(UL, n), rtol=1e-12, atol=1e-12)
        F2 = oracle.riemann("roe", UL, UR, -n)  # everything moves against -n -> right state
        assert np.allclose(F2, oracle.inviscid_flux(UR, -n), rtol=1e-12, atol=1e-12)
        assert c > 0


def test_stationary_contact():
    n = unit(rng)
    p = 1.7
    UL, UR = cons(1.0, [0, 0, 0], p), cons(2.5, [0, 0, 0], p)
    Froe = oracle.riemann("roe", UL, UR, n)
    assert np.allclose(Froe, [0, *(p * n), 0], atol=1e-14)
    Fr = oracle.riemann("rusanov", UL, UR, n)
    cmax = max(math.sqrt(G * p / 1.0), math.sqrt(G * p / 2.5))
    assert abs(Fr[0] - (-0.5 * cmax * (2.5 - 1.0))) < 1e-14
    assert np.allclose(Fr[1:4], p * n, atol=1e-14)
    assert abs(Fr[4]) < 1e-14  # E is equal on both sides


def test_rusanov_more_dissipative_than_roe_on_acoustic_jump():
    # Rusanov damps every wave at the fastest speed, Roe at each wave's own speed: the
    # dissipation Rusanov adds over Roe is a non-negative multiple of the jump in each wave.
    n = np.array([1.0, 0, 0])
    UL = cons(1.0, [0.2, 0, 0], 1.0)
    UR = cons(1.0, [0.2, 0, 0], 1.0 + 1e-6)
    Fc = 0.5 * (oracle.inviscid_flux(UL, n) + oracle.inviscid_flux(UR, n))
    dR = Fc - oracle.riemann("rusanov", UL, UR, n)
    dA = Fc - oracle.riemann("roe", UL, UR, n)
    assert dR[4] > dA[4] > 0


def test_viscous_simple_shear():
    mu, a, rho, u0 = 0.01, 0.7, 1.3, 0.4
    U = cons(rho, [u0, 0, 0], 1.0)
    Gr = np.zeros((3, 5))
    Gr[1, 1] = rho * a            # d(rho u)/dy
    Gr[1, 4] = rho * u0 * a       # d(E)/dy with E = p/(g-1) + rho u^2/2 and uniform p, rho
    Fv = oracle.viscous_flux(U, Gr, mu)
    expect = np.zeros((3, 5))
    expect[0, 2] = mu * a       # tau_xy
    expect[1, 1] = mu * a       # tau_yx
    expect[1, 4] = mu * a * u0  # tau_yx u
    assert np.allclose(Fv, expect, atol=1e-15)


def test_viscous_dilatation_and_conduction():
    mu, a, rho = 0.02, 0.3, 1.0
    U = cons(rho, [0, 0, 0], 2.0)
    Gr = np.zeros((3, 5))
    Gr[0, 1] = rho * a  # du/dx = a at u = 0
    Fv = oracle.viscous_flux(U, Gr, mu)
    assert abs(Fv[0, 1] - 4.0 / 3.0 * mu * a) < 1e-15
    assert abs(Fv[1, 2] + 2.0 / 3.0 * mu * a) < 1e-15
    assert abs(Fv[2, 3] + 2.0 / 3.0 * mu * a) < 1e-15
    # conduction: dE/dx = b with rho const and u = 0 -> dT'/dx = (g-1) b for T' = p/rho;
    # heat flux coefficient c_p mu / Pr with c_p = g R/(g-1) gives mu g/Pr * b in energy.
    b = 0.9
    Gr = np.zeros((3, 5))
    Gr[0, 4] = b
    Fv = oracle.viscous_flux(U, Gr, mu, prandtl=0.72)
    assert abs(Fv[0, 4] - mu * G / 0.72 * b) < 1e-14
    assert np.allclose(Fv[1:, :], 0) and np.allclose(Fv[0, :4], 0)


def test_viscous_rotational_invariance():
    r = np.random.default_rng(5)
    for _ in range(10):
        U, Q = random_state(r), rotation(r)
        Gr = r.normal(size=(3, 5))
        Fv = oracle.viscous_flux(U, Gr, 0.05)
        # rotate: x' = Q x; U' = (rho, Q m, E); d/dx'_i = Q_ij d/dx_j
        Ur = rot_state(Q, U)
        Gq = Q @ Gr                      # rotate the derivative direction
        Gq[:, 1:4] = Gq[:, 1:4] @ Q.T     # rotate the momentum components
        Fr = oracle.viscous_flux(Ur, Gq, 0.05)
        expect = Q @ Fv
        expect[:, 1:4] = expect[:, 1:4] @ Q.T
        assert np.allclose(Fr, expect, rtol=1e-12, atol=1e-12)
