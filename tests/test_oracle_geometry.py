"""Pins for the oracle's mesh handling and metric terms (Eq. (1): J_ij = dx_i/dxi_j, and the
transformed fluxes |J| J^-1 F).

* affine and trilinear elements: the curl-form metrics equal |J| J^-1 computed here from the
  closed-form map (exact for trilinear maps once p >= 2);
* the discrete metric identity sum_n D_n Ja^n_i = 0 holds on a curved isoparametric mesh;
* face matching: matched face points coincide in space and the two sides' normals are opposite;
* the quadrature volume of a conforming trilinear periodic mesh equals the box volume.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs


def gl(p):
    return np.polynomial.legendre.leggauss(p + 1)


def lagrange_deriv_matrix(x):
    """D[a, b] = l_b'(x_a) built from numpy polynomials (independent of the oracle)."""
    n = len(x)
    D = np.zeros((n, n))
    for b in range(n):
        others = np.delete(x, b)
        poly = np.polynomial.Polynomial.fromroots(others)
        poly = poly / poly(x[b])
        D[:, b] = poly.deriv()(x)
    return D


def trilinear_jacobian(Xc, xi):
    """Xc [2,2,2,3] corner coords indexed [k][j][i]; xi [N,3] -> J [N,3,3] with J[c,k]=dx_c/dxi_k."""
    N = xi.shape[0]
    J = np.zeros((N, 3, 3))
    phi = lambda b, t: (1 - t) / 2 if b == 0 else (1 + t) / 2
    dphi = lambda b, t: -0.5 * np.ones_like(t) if b == 0 else 0.5 * np.ones_like(t)
    for k in range(2):
        for j in range(2):
            for i in range(2):
                X = Xc[k, j, i]
                a, b, c = xi[:, 0], xi[:, 1], xi[:, 2]
                J[:, :, 0] += np.outer(dphi(i, a) * phi(j, b) * phi(k, c), X)
                J[:, :, 1] += np.outer(phi(i, a) * dphi(j, b) * phi(k, c), X)
                J[:, :, 2] += np.outer(phi(i, a) * phi(j, b) * dphi(k, c), X)
    return J


def sol_xi(p):
    x = gl(p)[0]
    k, j, i = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)


@pytest.mark.parametrize("p", [1, 3])
def test_affine_metrics_are_cofactor(p):
    m = inputs.box_mesh(3, q=1)
    A = np.array([[1.2, 0.3, -0.1], [0.1, 0.9, 0.25], [-0.2, 0.15, 1.1]])
    m.elem_nodes = m.elem_nodes @ A.T + np.array([0.3, -0.2, 0.5])
    o = oracle.Oracle(m, p)
    Ja, dJ, Nf, Jf = o.geometry()
    h = 2 * np.pi / 3
    J = A * (h / 2)  # dx_c/dxi_k
    expect = np.linalg.det(J) * np.linalg.inv(J)  # [n, i] = |J| dxi_n/dx_i
    assert np.allclose(Ja, expect, atol=1e-13)
    assert np.allclose(dJ, np.linalg.det(J), rtol=1e-13)
    # outward normal of face (d, s) is s * Ja^d
    for f in range(6):
        d, s = f // 2, (1 if f % 2 else -1)
        assert np.allclose(Nf[:, f], s * expect[d], atol=1e-13)
    assert np.allclose(Jf, np.linalg.det(J), rtol=1e-13)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_trilinear_metrics_exact(p):
    rng = np.random.default_rng(p)
    m = inputs.box_mesh(3, q=1)
    m.elem_nodes = m.elem_nodes + rng.uniform(-0.25, 0.25, size=m.elem_nodes.shape)
    o = oracle.Oracle(m, p)
    Ja, dJ, _, _ = o.geometry()
    xi = sol_xi(p)
    for e in range(m.n_elem):
        Xc = m.elem_nodes[e].reshape(2, 2, 2, 3)
        J = trilinear_jacobian(Xc, xi)
        det = np.linalg.det(J)
        expect = det[:, None, None] * np.linalg.inv(J)
        assert np.allclose(Ja[e], expect, atol=1e-12)
        assert np.allclose(dJ[e], det, atol=1e-12)
    # sol coords: trilinear map of the GL points
    X = o.sol_coords()
    e = 3
    Xc = m.elem_nodes[e].reshape(2, 2, 2, 3)
    phi = lambda b, t: (1 - t) / 2 if b == 0 else (1 + t) / 2
    ref = sum(np.outer(phi(i, xi[:, 0]) * phi(j, xi[:, 1]) * phi(k, xi[:, 2]), Xc[k, j, i])
              for k in range(2) for j in range(2) for i in range(2))
    assert np.allclose(X[e].T, ref, atol=1e-13)


@pytest.mark.parametrize("p,q", [(3, 3), (4, 2), (7, 7)])
def test_discrete_metric_identity_curved(p, q):
    n = 3
    m = inputs.box_mesh(n, q=q, curve_amp=0.05)
    o = oracle.Oracle(m, p)
    Ja, dJ, _, _ = o.geometry()
    D = lagrange_deriv_matrix(gl(p)[0])
    N = p + 1
    Jr = Ja.reshape(m.n_elem, N, N, N, 3, 3)  # [e, k, j, i, n, i]
    div = (np.einsum("ai,ekjin->ekjan", D, Jr[..., 0, :])
           + np.einsum("aj,ekjin->ekain", D, Jr[..., 1, :])
           + np.einsum("ak,ekjin->eajin", D, Jr[..., 2, :]))
    assert np.abs(div).max() < 1e-12 * max(1.0, np.abs(Ja).max())
    assert np.all(dJ > 0)


def face_points(X, p, f):
    """Interpolate a solution-point field X [C, Ns] to face f's points [C, Nfp] (numpy)."""
    x = gl(p)[0]
    N = p + 1
    d, s = f // 2, f % 2
    ell = np.array([np.prod([((1.0 if s else -1.0) - x[m]) / (x[b] - x[m])
                             for m in range(N) if m != b]) for b in range(N)])
    Xr = X.reshape(X.shape[0], N, N, N)  # [C, k, j, i]
    if d == 0:
        out = np.einsum("c,xkjc->xkj", ell, Xr)  # over i -> [C, k(t2), j(t1)]
    elif d == 1:
        out = np.einsum("c,xkci->xki", ell, Xr)  # over j -> [C, k(t2), i(t1)]
    else:
        out = np.einsum("c,xcji->xji", ell, Xr)  # over k -> [C, j(t2), i(t1)]
    return out.reshape(X.shape[0], N * N)  # a (t1) fastest


@pytest.mark.parametrize("scramble", [False, True])
def test_face_matching_and_watertight_normals(scramble):
    p = 3
    m = inputs.box_mesh(3, q=3, curve_amp=0.05)
    if scramble:
        m, _ = inputs.scramble_mesh(m, seed=7)
    o = oracle.Oracle(m, p)
    nbr, nface, owner, perm = o.connectivity()
    X = o.sol_coords()
    _, _, Nf, _ = o.geometry()
    L = 2 * np.pi
    for e in range(m.n_elem):
        for f in range(6):
            en, fn = nbr[e, f], nface[e, f]
            assert owner[e, f] + owner[en, fn] == 1
            a = face_points(X[e], p, f)
            b = face_points(X[en], p, fn)[:, perm[e, f]]
            diff = a - b
            diff -= L * np.round(diff / L)  # periodic images
            assert np.abs(diff).max() < 1e-12
            assert np.allclose(Nf[e, f], -Nf[en, fn][perm[e, f]], atol=1e-13)


def test_trilinear_periodic_volume():
    rng = np.random.default_rng(11)
    n = 3
    m = inputs.box_mesh(n, q=1)
    # displace every (periodically merged) vertex consistently
    disp = rng.uniform(-0.15, 0.15, size=(n ** 3, 3))
    corner_lattice_to_node = [0, 1, 3, 2, 4, 5, 7, 6]  # VTK corner -> tensor node index
    for e in range(m.n_elem):
        for c in range(8):
            m.elem_nodes[e, corner_lattice_to_node[c]] += disp[m.elem_vert[e, c]]
    p = 2
    o = oracle.Oracle(m, p)
    _, dJ, _, _ = o.geometry()
    w = gl(p)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    assert abs((dJ * W).sum() - (2 * np.pi) ** 3) < 1e-10


def test_rejects_bad_meshes():
    m = inputs.box_mesh(3, q=1)
    bad = inputs.Mesh(elem_vert=m.elem_vert[:-1].copy(), elem_nodes=m.elem_nodes[:-1].copy(), q=1)
    with pytest.raises(RuntimeError, match="unpaired"):
        oracle.Oracle(bad, 2)
    inv = inputs.Mesh(elem_vert=m.elem_vert.copy(), elem_nodes=m.elem_nodes.copy(), q=1)
    inv.elem_nodes[0, :, 0] *= -1.0  # mirror element 0: negative Jacobian
    with pytest.raises(RuntimeError, match="Jacobian"):
        oracle.Oracle(inv, 2)
