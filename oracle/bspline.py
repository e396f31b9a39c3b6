"""Univariate B-splines (Sec. 5.1: open knot vector, Cox-de Boor recursion with
the convention 0/0 = 0) and the Gauss-Legendre rule used for all integrals.

Readings:
* Knots: open and uniform with simple interior knots, i.e. splines of maximal
  regularity C^{p-1} (Sec. 6 uses only maximal regularity).
* Quadrature (the paper is silent): p+1 Gauss-Legendre points per element per
  direction.  The rule itself comes from ``numpy.polynomial.legendre.leggauss``.
* Derivatives (not written in the paper): the standard de Boor identity
  b'_{i,p} = p/(xi_{i+p}-xi_i) b_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) b_{i+1,p-1},
  again with 0/0 = 0.
"""
import numpy as np


def open_uniform_knots(n, p):
    """Open knot vector on [0,1] with n uniform elements (Sec. 5.1): p+1 copies
    of 0 and 1, interior knots i/n with multiplicity one.  Length n+2p+1, so
    m = n+p basis functions."""
    return np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])


def _ratio(num, den):
    """num/den with 0/0 = 0 (and x/0 = 0: happens only where the basis below is 0)."""
    shape = np.broadcast(num, den).shape
    num = np.broadcast_to(num, shape)
    den = np.broadcast_to(den, shape)
    out = np.zeros(shape)
    nz = den != 0
    out[nz] = num[nz] / den[nz]
    return out


def basis(knots, p, x, deriv=False):
    """Values (and, if ``deriv``, first derivatives) of all m = len(knots)-p-1
    B-splines of degree p at points x, by the Cox-de Boor recursion of Sec. 5.1.

    Degree 0 uses the half-open spans [xi_i, xi_{i+1}) as printed, so points
    must lie in [0,1); Gauss points always do.  Returns arrays [len(x), m]."""
    x = np.asarray(x, dtype=np.float64)
    xi = np.asarray(knots, dtype=np.float64)
    nk = len(xi)
    # degree 0
    b = ((xi[None, :-1] <= x[:, None]) & (x[:, None] < xi[None, 1:])).astype(np.float64)
    prev = None
    for q in range(1, p + 1):
        cnt = nk - q - 1
        left = _ratio(x[:, None] - xi[None, :cnt], xi[None, q:q + cnt] - xi[None, :cnt])
        right = _ratio(xi[None, q + 1:q + 1 + cnt] - x[:, None],
                       xi[None, q + 1:q + 1 + cnt] - xi[None, 1:1 + cnt])
        prev = b
        b = left * b[:, :cnt] + right * b[:, 1:cnt + 1]
    if not deriv:
        return b
    if p == 0:
        return b, np.zeros_like(b)
    m = nk - p - 1
    cl = _ratio(np.full(m, float(p)), xi[p:p + m] - xi[:m])
    cr = _ratio(np.full(m, float(p)), xi[p + 1:p + 1 + m] - xi[1:1 + m])
    d = cl[None, :] * prev[:, :m] - cr[None, :] * prev[:, 1:m + 1]
    return b, d


def gauss_rule(nq):
    """nq-point Gauss-Legendre rule on [0,1] (library routine, rescaled)."""
    t, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (t + 1.0), 0.5 * w


def quadrature_1d(n, p, nq=None):
    """Global 1-D quadrature on the n uniform elements of [0,1]: points [n*nq],
    weights [n*nq], ordered element by element, nq = p+1 by default."""
    nq = p + 1 if nq is None else nq
    t, w = gauss_rule(nq)
    e = np.arange(n)[:, None]
    xq = ((e + t[None, :]) / n).ravel()
    wq = np.broadcast_to(w[None, :] / n, (n, nq)).ravel().copy()
    return xq, wq


def tables_1d(n, p, nq=None):
    """Basis values B [Q, m] and derivatives D [Q, m] at the global 1-D Gauss
    points, plus the points and weights."""
    knots = open_uniform_knots(n, p)
    xq, wq = quadrature_1d(n, p, nq)
    B, D = basis(knots, p, xq, deriv=True)
    return xq, wq, B, D
