"""Pins for the oracle's source term S of Eq. (3), read as a constant body force g per unit
mass ("body forcing" is among the solver's physical models, section "ZFR Framework"):
S = (0, rho g, m . g).

* a uniform state has zero flux divergence, so its residual is exactly S;
* a uniform state accelerated by g stays uniform, with m(t) = m0 + rho g t and
  E(t) = E0 + (m0 . g) t + rho |g|^2 t^2 / 2: any fourth-order Runge-Kutta method integrates
  this quadratic in t exactly (to rounding);
* mass is conserved and the momentum source integrates to g times the mass.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs as I

G = np.array([0.3, -0.2, 0.1])


def test_uniform_state_residual_is_source():
    m = I.box_mesh(3, q=3, curve_amp=0.05, curve_mode="mixed")
    o = oracle.Oracle(m, 3, mu=0.01, flux="roe")
    U = I.state_from_coords(o.sol_coords(), I.freestream_state)
    o.set_body_force(G)
    R = o.residual(U)
    S = np.zeros_like(U)
    S[:, 1:4] = U[:, 0:1] * G[None, :, None]
    S[:, 4] = np.einsum("eis,i->es", U[:, 1:4], G)
    assert np.abs(R - S).max() < 1e-9  # the freestream floor on the curved mesh


@pytest.mark.parametrize("scheme", ["rk4", "lsrk45", "ssprk104"])
def test_uniformly_accelerated_state_exact(scheme):
    m = I.box_mesh(3, q=1)
    o = oracle.Oracle(m, 2, mu=0.01, flux="rusanov")
    U0 = I.state_from_coords(o.sol_coords(), I.freestream_state)
    o.set_body_force(G)
    dt, n = 0.01, 8  # inside every scheme's stability limit for this mesh
    U = o.rk_step(U0, dt, scheme, n)
    t = dt * n
    rho = U0[:, 0]
    m0 = U0[:, 1:4]
    exact = U0.copy()
    exact[:, 1:4] = m0 + rho[:, None] * G[None, :, None] * t
    exact[:, 4] = U0[:, 4] + np.einsum("eis,i->es", m0, G) * t + 0.5 * rho * (G @ G) * t * t
    assert np.abs(U - exact).max() < 1e-11


def test_source_conservation():
    p = 3
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    o = oracle.Oracle(m, p, mu=0.01, flux="roe")
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=3, amp=0.01)
    _, dJ, _, _ = o.geometry()
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    R0 = o.residual(U)
    o.set_body_force(G)
    R = o.residual(U)
    tot = np.einsum("evs,es,s->v", R - R0, dJ, W)
    mass = np.einsum("es,es,s->", U[:, 0], dJ, W)
    assert abs(tot[0]) < 1e-14
    assert np.allclose(tot[1:4], G * mass, rtol=1e-12)
    o.set_body_force(np.zeros(3))
    assert np.array_equal(o.residual(U), R0)
