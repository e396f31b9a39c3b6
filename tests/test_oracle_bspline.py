"""Pins of the oracle's univariate toolkit (Sec. 5.1) against library routines
and closed forms."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [1, 2, 5, 7])
def test_cox_de_boor_matches_scipy(p, n):
    kn = bspline.open_uniform_knots(n, p)
    x = np.random.default_rng(1).uniform(0, 1, 50)
    B, D = bspline.basis(kn, p, x, deriv=True)
    m = n + p
    assert B.shape == (50, m)
    for i in range(m):
        c = np.zeros(m)
        c[i] = 1.0
        s = BSpline(kn, c, p, extrapolate=False)
        np.testing.assert_allclose(B[:, i], np.nan_to_num(s(x)), atol=1e-14)
        if p > 0:
            np.testing.assert_allclose(D[:, i], np.nan_to_num(s.derivative()(x)), atol=1e-11)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_partition_of_unity(p):
    # eq. partition_unity: sum_i b_{i,p}(x) = 1 on (0, 1); derivatives sum to 0
    kn = bspline.open_uniform_knots(6, p)
    x = np.linspace(0.001, 0.999, 77)
    B, D = bspline.basis(kn, p, x, deriv=True)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11)
    assert np.all(B >= 0)


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5])
def test_gauss_rule_exactness(nq):
    t, w = bspline.gauss_rule(nq)
    for deg in range(2 * nq):
        assert abs(np.sum(w * t ** deg) - 1.0 / (deg + 1)) < 1e-14
    assert abs(np.sum(w * t ** (2 * nq)) - 1.0 / (2 * nq + 1)) > 1e-8


def test_quadrature_points_inside_elements():
    xq, wq = bspline.quadrature_1d(5, 3)
    assert len(xq) == 20 and abs(wq.sum() - 1.0) < 1e-14
    e = np.floor(xq * 5).astype(int)
    np.testing.assert_array_equal(e, np.repeat(np.arange(5), 4))
