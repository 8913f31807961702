"""Pins for the oracle's isothermal no-slip walls (the channel meshes of the batched workload;
the paper lists boundary conditions among the solver's models without detail).

Reading: the wall face is owned by its element. Inviscid part: the Riemann flux against the
mirror state (rho, -m, E). Viscous part (BR2): the wall state U_w = (rho_L, 0, rho_L T_w/(gamma-1))
is the common state and the common gradient is one-sided, G_L + eta r_L with r_L the lifting
of U_w - U_L. Fixed independently of the oracle by:
* a fluid at rest at the wall temperature is steady (zero residual);
* the mirror flux is impermeable, so mass is conserved exactly with walls;
* the energy equation of a fluid at rest (E_t = nu E_xx) equals a textbook modal DG-BR2
  discretisation with Dirichlet values at both walls, built here from Legendre polynomials;
* a wall-parallel flow loses momentum to the walls and none along them;
* the element-subset mode agrees with the full residual.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs as I

G, PR = 1.4, 0.72
TW = 1.0 / (G * 0.01)  # p/rho of the Mach 0.1 reference state


def weights3(p):
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    return np.einsum("k,j,i->kji", w, w, w).ravel()


def channel(n=(3, 4, 3), q=1, curve=0.0):
    m = I.box_mesh(n, q=q, periodic=(True, False, True), curve_amp=curve, curve_mode="mixed")
    return m, I.boundary_tags(m)


def rest_state(X, T=TW):
    U = np.zeros((X.shape[0], 5, X.shape[2]))
    U[:, 0] = 1.0
    U[:, 4] = T / (G - 1)
    return U


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_rest_at_wall_temperature_is_steady(flux):
    m, tags = channel(curve=0.05, q=2)
    o = oracle.Oracle(m, 3, mu=0.01, flux=flux, bc_tag=tags, wall_T=TW)
    R = o.residual(rest_state(o.sol_coords()))
    assert np.abs(R).max() < 1e-10
    assert tags.sum() == 2 * 3 * 3  # two walls of 3 x 3 faces


def test_unpaired_face_without_tag_rejected():
    m, tags = channel()
    with pytest.raises(RuntimeError):
        oracle.Oracle(m, 2, mu=0.01)
    o = oracle.Oracle(m, 2, mu=0.01, bc_tag=tags)
    with pytest.raises(RuntimeError):
        o.set_viscous_scheme("ldg")


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_mass_conservation_with_walls(flux):
    p = 3
    m, tags = channel(n=(3, 4, 3), q=2, curve=0.05)
    o = oracle.Oracle(m, p, mu=0.01, flux=flux, bc_tag=tags, wall_T=TW)
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=4, amp=0.02)
    R = o.residual(U)
    _, dJ, _, _ = o.geometry()
    W = weights3(p)
    tot = np.einsum("es,es,s->", R[:, 0], dJ, W)
    mag = np.einsum("es,es,s->", np.abs(R[:, 0]), dJ, W)
    assert abs(tot) / mag < 1e-13


def dg_br2_heat_dirichlet(u_nodes, h, nu, eta, p, u_wall):
    """Textbook modal DG-BR2 for u_t = nu u_xx on n elements between two walls with u = u_wall:
    interior faces as in the periodic case; at a wall U^ = u_wall, the lifting is that of
    (u_wall - u_K) and the common gradient is one-sided, q^ = u_x + eta r at the element's end."""
    L = np.polynomial.legendre
    n = u_nodes.shape[0]
    xg, _ = L.leggauss(p + 1)
    V = L.legvander(xg, p)
    c = np.linalg.solve(V, u_nodes.T).T
    xq, wq = L.leggauss(p + 4)
    Pq = L.legvander(xq, p)
    dmode = [L.legder(np.eye(p + 1)[m]) if p > 0 else np.zeros(1) for m in range(p + 1)]
    dPq = np.stack([L.legval(xq, dm) for dm in dmode], 1)
    Pm, Pp = L.legvander(np.array([-1.0]), p)[0], L.legvander(np.array([1.0]), p)[0]
    dPm = np.array([L.legval(-1.0, dm) for dm in dmode])
    dPp = np.array([L.legval(1.0, dm) for dm in dmode])
    J = h / 2
    M = J * Pq.T @ (wq[:, None] * Pq)
    Minv = np.linalg.inv(M)
    uR, uL = c @ Pp, c @ Pm
    uhat_right = np.array([0.5 * (uR[K] + uL[K + 1]) if K < n - 1 else u_wall for K in range(n)])
    uhat_left = np.array([0.5 * (uL[K] + uR[K - 1]) if K > 0 else u_wall for K in range(n)])
    r_right = ((uhat_right - uR)[:, None] * Pp[None, :]) @ Minv.T
    r_left = ((uhat_left - uL)[:, None] * (-Pm)[None, :]) @ Minv.T
    gR = (c @ dPp) / J + eta * (r_right @ Pp)  # u_x + eta r_f at each element's right end
    gL = (c @ dPm) / J + eta * (r_left @ Pm)
    ut = np.zeros_like(c)
    for K in range(n):
        qhat_r = 0.5 * (gR[K] + gL[K + 1]) if K < n - 1 else gR[K]
        qhat_l = 0.5 * (gL[K] + gR[K - 1]) if K > 0 else gL[K]
        qK = (dPq @ c[K]) / J + Pq @ (r_right[K] + r_left[K])
        rhs = -nu * (dPq.T @ (wq * qK)) + nu * (Pp * qhat_r - Pm * qhat_l)
        ut[K] = Minv @ rhs
    return ut @ V.T


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_heat_between_walls_is_textbook_br2(p):
    rng = np.random.default_rng(p)
    n, Ly, mu, eta = 5, 2.0, 0.05, 6.0
    m = I.box_mesh((3, n, 3), lo=(0, 0, 0), hi=(1, Ly, 1), q=1, periodic=(True, False, True))
    tags = I.boundary_tags(m)
    N = p + 1
    Ew = TW / (G - 1)
    E_nodes = Ew + 0.5 * rng.normal(size=(n, N))
    U = np.zeros((m.n_elem, 5, N ** 3))
    U[:, 0] = 1.0
    for e in range(m.n_elem):
        je = (e // 3) % n  # element (ie, je, ke) has index ie + 3 (je + n ke)
        U[e, 4] = E_nodes[je][(np.arange(N ** 3) // N) % N]  # point i + N (j + N k): varies with j
    Rv = oracle.Oracle(m, p, mu=mu, flux="rusanov", bc_tag=tags, wall_T=TW).residual(U)
    R0 = oracle.Oracle(m, p, mu=0.0, flux="rusanov", bc_tag=tags, wall_T=TW).residual(U)
    d = (Rv - R0)[:, 4, :]
    # the line i = k = 0 through elements ie = ke = 0, along y
    fr = np.stack([d[3 * je, [j * N for j in range(N)]] for je in range(n)])
    nu = mu * G / PR
    dg = dg_br2_heat_dirichlet(E_nodes, Ly / n, nu, eta, p, Ew)
    assert np.abs(fr - dg).max() < 1e-9 * np.abs(dg).max(), np.abs(fr - dg).max()


def test_wall_friction_decelerates_parallel_flow():
    p = 3
    m, tags = channel(n=(3, 4, 3))
    o = oracle.Oracle(m, p, mu=0.01, flux="roe", bc_tag=tags, wall_T=TW)
    X = o.sol_coords()
    U = rest_state(X)
    U[:, 3] = 0.5  # uniform flow along z, parallel to the y walls
    U[:, 4] += 0.5 * 0.25
    R = o.residual(U)
    _, dJ, _, _ = o.geometry()
    W = weights3(p)
    mom = np.einsum("evs,es,s->v", R[:, 1:4], dJ, W)
    assert mom[2] < -1e-3          # drag along the flow
    assert abs(mom[0]) < 1e-12 * abs(mom[2])  # nothing along x
    # the elements next to a wall decelerate, the interior ones do not (uniform flow)
    je = (np.arange(m.n_elem) // 3) % 4
    Rz = np.einsum("es,es,s->e", R[:, 3], dJ, W)
    assert np.all(Rz[(je == 0) | (je == 3)] < 0)
    assert np.abs(Rz[(je == 1) | (je == 2)]).max() < 1e-10


def test_subset_with_walls():
    m, tags = channel(n=(3, 4, 3), q=2, curve=0.05)
    o = oracle.Oracle(m, 2, mu=0.01, flux="roe", bc_tag=tags)
    U = I.state_from_coords(o.sol_coords(), I.tgv_state)
    R = o.residual(U)
    act = np.array([0, 4, 17, 35, 20])
    os_ = oracle.Oracle(m, 2, mu=0.01, flux="roe", bc_tag=tags, active=act)
    assert np.array_equal(os_.residual(U), R[act])
