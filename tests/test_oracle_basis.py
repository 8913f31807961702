"""Pins for the oracle's 1-D basis (section "FR Algorithm", Eq. (2) and the choice of g).

* Gauss-Legendre points/weights against numpy's leggauss.
* GLL quadrature is exact for monomials up to degree 2N-1.
* D is exact on x^k for k <= p and its rows sum to zero; end interpolation is exact on x^k.
* The correction derivatives satisfy the DG lifting identity g'(xi_a) w_a = l_a(+-1): that is
  the statement that FR with g_DG equals a nodal collocated DG method.
"""
import numpy as np
import pytest

import oracle

PS = [0, 1, 2, 3, 4, 5, 6, 7]


@pytest.mark.parametrize("p", PS)
def test_gauss_legendre_matches_numpy(p):
    b = oracle.basis(p)
    x, w = np.polynomial.legendre.leggauss(p + 1)
    assert np.allclose(b["xs"], x, atol=1e-15, rtol=0)
    assert np.allclose(b["ws"], w, atol=1e-15, rtol=0)
    assert abs(b["ws"].sum() - 2.0) < 1e-14


@pytest.mark.parametrize("p", PS)
def test_gll_quadrature_exact(p):
    b = oracle.basis(p)
    N = max(p, 1)
    xg, wg = b["xg"], b["wg"]
    assert xg[0] == -1.0 and xg[-1] == 1.0
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(wg, xg ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", PS)
def test_derivative_and_end_interpolation_exact(p):
    b = oracle.basis(p)
    x = b["xs"]
    for k in range(p + 1):
        f = x ** k
        df = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.allclose(b["D"] @ f, df, atol=1e-12 * max(1, p) ** 2)
        assert abs(b["lm"] @ f - (-1.0) ** k) < 1e-13
        assert abs(b["lp"] @ f - 1.0) < 1e-13
    assert np.allclose(b["D"].sum(axis=1), 0.0, atol=1e-12)


@pytest.mark.parametrize("p", PS)
def test_correction_is_dg_lifting(p):
    # sum_a w_a g'(xi_a) v(xi_a) = v(+1) for every v of degree <= p holds for the Radau g_DG
    # choice and no other degree-(p+1) correction with g(-1)=0, g(1)=1.
    b = oracle.basis(p)
    assert np.allclose(b["gcR"] * b["ws"], b["lp"], atol=1e-13)
    assert np.allclose(b["gcL"] * b["ws"], b["lm"], atol=1e-13)
    # interpolating g_R' to xi = 1 gives g_R'(1) = (p+1)^2 / 2
    assert abs(b["lp"] @ b["gcR"] - (p + 1) ** 2 / 2) < 1e-11


@pytest.mark.parametrize("p", [3, 7])
def test_precisions_agree(p):
    a = oracle.basis(p, "f64")
    b = oracle.basis(p, "ld")
    f = oracle.basis(p, "f32")
    for k in ("xs", "ws", "D", "gcR", "xg"):
        assert np.allclose(a[k], b[k], atol=1e-14 * max(1.0, np.abs(b[k]).max()))
        assert np.allclose(f[k], b[k], atol=1e-5 * max(1.0, np.abs(b[k]).max()))
