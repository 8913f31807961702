"""Host-side pieces of the closure pipeline: the fine-to-coarse filter and the random-phase
initial spectra (no GPU).

* the 1-D restriction reproduces every polynomial of the coarse degree exactly, is the L2
  projection (the residual of any field is orthogonal to the coarse polynomials), and the 3-D
  filter preserves each coarse element's mean (a conservative filter);
* the spectrum state is divergence free as a continuous field (checked on its Fourier
  description), has the requested mean kinetic energy, and is laid out consistently with the
  solution-point coordinates.
"""
import numpy as np

from paper_2308_06605_amd import closure as C
from paper_2308_06605_amd import inputs as I


def test_restriction_reproduces_coarse_polynomials():
    pc, pf, r = 3, 7, 2
    Rm = C.restriction_1d(pc, pf, r)
    xf = np.polynomial.legendre.leggauss(pf + 1)[0]
    xi = np.concatenate([-1.0 + (2 * k + xf + 1.0) / r for k in range(r)])
    xc = np.polynomial.legendre.leggauss(pc + 1)[0]
    for deg in range(pc + 1):
        c = np.random.default_rng(deg).normal(size=deg + 1)
        assert np.allclose(Rm @ np.polynomial.polynomial.polyval(xi, c), np.polynomial.polynomial.polyval(xc, c),
                           atol=1e-13)


def test_restriction_is_l2_projection():
    pc, pf, r = 3, 7, 2
    Rm = C.restriction_1d(pc, pf, r)
    xf, wf = np.polynomial.legendre.leggauss(pf + 1)
    xi = np.concatenate([-1.0 + (2 * k + xf + 1.0) / r for k in range(r)])
    w = np.tile(wf, r) / r
    xc = np.polynomial.legendre.leggauss(pc + 1)[0]
    f = np.sin(3 * xi) + xi ** 5  # piecewise data of higher degree
    proj = Rm @ f
    # the projection's polynomial, evaluated at the fine points through Lagrange interpolation
    Lc = np.stack([np.prod([(xi - xc[m]) / (xc[b] - xc[m]) for m in range(pc + 1) if m != b], axis=0)
                   for b in range(pc + 1)], axis=1)
    resid = f - Lc @ proj
    for deg in range(pc + 1):
        assert abs((w * resid * xi ** deg).sum()) < 1e-13


def test_filter_preserves_element_means():
    pf, pc = 5, 2
    mf = I.box_mesh(6, q=1)
    rng = np.random.default_rng(0)
    Uf = rng.normal(size=(mf.n_elem, 5, (pf + 1) ** 3))
    Uc = C.restrict(Uf, mf.shape, pf, pc, 2)
    Wf, Wc = C.quad_weights(pf), C.quad_weights(pc)
    mean_f = np.einsum("evs,s->ev", Uf, Wf).reshape(3, 2, 3, 2, 3, 2, 5).sum(axis=(1, 3, 5)).reshape(27, 5) / 8
    mean_c = np.einsum("evs,s->ev", Uc, Wc)
    assert np.allclose(mean_f, mean_c, atol=1e-12)
    # idempotent on a field that is already coarse: restrict(prolong(Uc)) == Uc
    xf = np.polynomial.legendre.leggauss(pf + 1)[0]
    xc = np.polynomial.legendre.leggauss(pc + 1)[0]
    xi = np.concatenate([-1.0 + (2 * k + xf + 1.0) / 2 for k in range(2)])
    Lc = np.stack([np.prod([(xi - xc[m]) / (xc[b] - xc[m]) for m in range(pc + 1) if m != b], axis=0)
                   for b in range(pc + 1)], axis=1).reshape(2, pf + 1, pc + 1)
    U3 = Uc.reshape(3, 3, 3, 5, pc + 1, pc + 1, pc + 1)  # cz cy cx v c b a
    # fine value at element (2cz+rz, 2cy+ry, 2cx+rx), point (k, j, i)
    P = np.einsum("Rkc,Sjb,Tia,zyxvcba->zRySxTvkji", Lc, Lc, Lc, U3)
    Ufine = P.reshape(216, 5, (pf + 1) ** 3)
    assert np.allclose(C.restrict(Ufine, mf.shape, pf, pc, 2), Uc, atol=1e-12)


def test_spectrum_state():
    import oracle

    p = 3
    m = I.box_mesh(4, q=1)
    U = I.random_spectrum_state(m, p, seed=3, k0=2.0)
    X = oracle.Oracle(m, p).sol_coords()
    # layout: the grid helpers place the axis coordinates where the solution points are
    ax = I.box_axis_points(m, p)
    Z, Y, Xg = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    assert np.allclose(I.grid_to_state_layout(np.stack([Xg, Y, Z]), m.shape, p), X)
    assert abs(C.kinetic_energy(U, p) - 0.125) < 1e-12
    assert np.all(U[:, 0] == 1.0)
    # reproducible, and different seeds differ
    assert np.array_equal(U, I.random_spectrum_state(m, p, seed=3, k0=2.0))
    assert not np.allclose(U, I.random_spectrum_state(m, p, seed=4, k0=2.0))


def test_spectrum_state_divergence_free_on_fine_grid():
    """On a grid fine enough to resolve every mode, the discrete divergence is small against
    the gradient: the continuous field is divergence free."""
    import oracle

    p = 7
    m = I.box_mesh(4, q=1)
    U = I.random_spectrum_state(m, p, seed=1, k0=2.0, kmax=4)
    f = oracle.Oracle(m, p).sgs_features(U)
    # features: ..., th / sqrt(s2), th2 / s2 (volume averages of div u and its square)
    assert np.abs(f[:, -1]).max() < 1e-6


def test_stress_target_zero_for_resolved_fields():
    """A fine field that is a polynomial of the coarse degree on each coarse element has no
    sub-grid stress, so its target eddy viscosity is zero; an unresolved field gets a positive
    one in a share of the elements."""
    C.configure((6, 5), (3, 2))
    try:
        mf = I.box_mesh(6, q=1)
        ax = I.box_axis_points(mf, 5)
        Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        # linear velocity (products are quadratic: inside the coarse degree 2)
        vel = np.stack([0.3 * Y - 0.1 * Z, 0.2 * X, -0.4 * X + 0.1 * Y])
        U = np.zeros((216, 5, 216))
        U[:, 0] = 1.0
        U[:, 1:4] = I.grid_to_state_layout(vel, mf.shape, 5)
        U[:, 4] = 100.0
        nu = C.stress_target(U, mf.shape, 2 * np.pi / 3)
        assert np.abs(nu).max() < 1e-12
        U2 = I.random_spectrum_state(mf, 5, seed=1, k0=2.0, kmax=4)
        nu2 = C.stress_target(U2, mf.shape, 2 * np.pi / 3)
        assert np.all(nu2 >= 0) and (nu2 > 0).mean() > 0.2
    finally:
        C.configure((32, 7), (16, 3))
