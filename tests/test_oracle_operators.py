"""Pins of the oracle's mass and stiffness matrices (eq. mass_matrix, K of
eq. mp with omega = 1) against closed forms, Kronecker identities, library
integration and brute force."""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import quad
from scipy.interpolate import BSpline

from oracle import bspline, operators
from paper_2102_11536_amd import workloads


def eulerian(nn, kk):
    # number of permutations of nn elements with kk ascents (recurrence)
    A = [[0] * (nn + 1) for _ in range(nn + 1)]
    A[0][0] = 1
    for a in range(1, nn + 1):
        for b in range(a):
            A[a][b] = (b + 1) * A[a - 1][b] + (a - b) * (A[a - 1][b - 1] if b else 0)
    return A[nn][kk]


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_1d_mass_interior_rows_are_eulerian(p):
    # Interior rows of the uniform univariate mass matrix: h * A(2p+1, j) / (2p+1)!
    n = 4 * p + 4
    M = operators.parametric_mass_1d(n, p)
    i = n // 2
    row = M[i, i - p:i + p + 1] * n
    ref = np.array([eulerian(2 * p + 1, j) for j in range(2 * p + 1)], float) / factorial(2 * p + 1)
    np.testing.assert_allclose(row, ref, rtol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_1d_mass_vs_scipy_quad(p):
    n = 3
    kn = bspline.open_uniform_knots(n, p)
    m = n + p
    M = operators.parametric_mass_1d(n, p)
    K = operators.parametric_stiffness_1d(n, p)
    fs = []
    for i in range(m):
        c = np.zeros(m)
        c[i] = 1
        fs.append(BSpline(kn, c, p))
    brk = list(np.arange(1, n) / n)
    for i in range(m):
        for j in range(m):
            v = quad(lambda x: fs[i](x) * fs[j](x), 0, 1, points=brk, epsabs=1e-15, epsrel=1e-13)[0]
            assert abs(M[i, j] - v) < 1e-13
            dv = quad(lambda x: fs[i].derivative()(x) * fs[j].derivative()(x), 0, 1,
                      points=brk, epsabs=1e-13, epsrel=1e-12)[0]
            assert abs(K[i, j] - dv) < 1e-10 * max(1, abs(dv))


@pytest.mark.parametrize("dim,p,n", [(2, 1, 3), (2, 2, 4), (2, 4, 2), (3, 2, 2), (3, 3, 3)])
def test_identity_map_kron_structure(dim, p, n):
    # identity map: M = Mz (x) My (x) Mx and K = sum of Khat in one slot
    sp_ = operators.Space(n, p, dim)
    ctrl = workloads.identity_ctrl(n, p, dim)
    M, K = operators.assemble(sp_, ctrl)
    Mh = operators.parametric_mass_1d(n, p)
    Kh = operators.parametric_stiffness_1d(n, p)
    Mref = Mh
    for _ in range(dim - 1):
        Mref = np.kron(Mh, Mref)
    Kref = 0
    for a in range(dim):
        t = np.ones((1, 1))
        for b in range(dim):
            t = np.kron(Kh if b == a else Mh, t)
        Kref = Kref + t
    np.testing.assert_allclose(M.toarray(), Mref, atol=1e-15)
    np.testing.assert_allclose(K.toarray(), Kref, atol=1e-12)


def test_affine_map_scaling_3d():
    # x = diag(s) xi + c:  M = s1 s2 s3 Mhat,  K = s1s2s3 * sum_a Khat_a / s_a^2
    n, p, s = 2, 2, np.array([2.0, 0.5, 3.0])
    sp_ = operators.Space(n, p, 3)
    ctrl = workloads.identity_ctrl(n, p, 3) * s[None, :] + np.array([1.0, -2.0, 0.25])
    M, K = operators.assemble(sp_, ctrl)
    Mh = operators.parametric_mass_1d(n, p)
    Kh = operators.parametric_stiffness_1d(n, p)
    vol = np.prod(s)
    Mref = vol * np.kron(Mh, np.kron(Mh, Mh))
    Kref = vol * (np.kron(Mh, np.kron(Mh, Kh)) / s[0] ** 2 + np.kron(Mh, np.kron(Kh, Mh)) / s[1] ** 2
                  + np.kron(Kh, np.kron(Mh, Mh)) / s[2] ** 2)
    np.testing.assert_allclose(M.toarray(), Mref, atol=1e-14)
    np.testing.assert_allclose(K.toarray(), Kref, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_deformed_map_invariants(dim):
    n, p = 3, 2
    sp_ = operators.Space(n, p, dim)
    ctrl = workloads.deformed_cube_ctrl(n, p, dim=dim)
    M, K = operators.assemble(sp_, ctrl)
    Md, Kd = M.toarray(), K.toarray()
    np.testing.assert_allclose(Md, Md.T, atol=1e-15)
    np.testing.assert_allclose(Kd, Kd.T, atol=1e-13)
    # gradient of a constant vanishes (partition of unity): K 1 = 0
    assert np.max(np.abs(Kd @ np.ones(len(Kd)))) < 1e-12
    # mass of the constant = volume = sum of the quadrature weights w|J|
    _, _, W, _ = operators.geometry_factors(sp_, ctrl)
    assert abs(np.ones(len(Md)) @ Md @ np.ones(len(Md)) - W.sum()) < 1e-13
    # coordinate functions are in the space: K-energy of x_c is the volume
    for c in range(dim):
        xc = ctrl[:, c]
        assert abs(xc @ Kd @ xc - W.sum()) < 1e-11
    assert np.all(np.linalg.eigvalsh(Md) > 0)


def test_brute_force_pointwise_3d():
    # M and K entry by entry with scipy's B-splines and explicit loops
    n, p, dim = 2, 2, 3
    sp_ = operators.Space(n, p, dim)
    ctrl = workloads.deformed_cube_ctrl(n, p, dim=dim)
    M, K = operators.assemble(sp_, ctrl)
    kn = bspline.open_uniform_knots(n, p)
    m = n + p
    fs = []
    for i in range(m):
        c = np.zeros(m)
        c[i] = 1
        fs.append(BSpline(kn, c, p))
    t, w = np.polynomial.legendre.leggauss(p + 1)
    pts = [((e + 0.5 * (tt + 1)) / n, 0.5 * ww / n) for e in range(n) for tt, ww in zip(t, w)]
    nd = m ** 3
    Mb = np.zeros((nd, nd))
    Kb = np.zeros((nd, nd))
    val = lambda i, x: float(fs[i](x))
    der = lambda i, x: float(fs[i].derivative()(x))
    for (x, wx) in pts:
        for (y, wy) in pts:
            for (z, wz) in pts:
                B = np.zeros(nd)
                dB = np.zeros((nd, 3))
                for iz in range(m):
                    for iy in range(m):
                        for ix in range(m):
                            g = ix + m * iy + m * m * iz
                            B[g] = val(ix, x) * val(iy, y) * val(iz, z)
                            dB[g] = [der(ix, x) * val(iy, y) * val(iz, z),
                                     val(ix, x) * der(iy, y) * val(iz, z),
                                     val(ix, x) * val(iy, y) * der(iz, z)]
                J = ctrl.T @ dB  # J[c, a]
                dj = np.linalg.det(J)
                grad = dB @ np.linalg.inv(J)  # rows: J^{-T} gradhat
                wq = wx * wy * wz * abs(dj)
                Mb += wq * np.outer(B, B)
                Kb += wq * grad @ grad.T
    np.testing.assert_allclose(M.toarray(), Mb, atol=1e-14)
    np.testing.assert_allclose(K.toarray(), Kb, atol=1e-12)


def test_1d_lowest_eigenvalue_tends_to_pi_squared():
    # -u'' = lam u on (0,1) with u(0)=u(1)=0: lam_min = pi^2
    errs = []
    for n in (4, 8, 16):
        sp_ = operators.Space((n,), 3)
        ctrl = workloads.identity_ctrl((n,), 3, 1)
        M, K = operators.free_operators(sp_, ctrl)
        lam = sla.eigh(K.toarray(), M.toarray(), eigvals_only=True)[0]
        errs.append(abs(lam - np.pi ** 2))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 1e-6


def test_sampled_rows_equal_assembled_rows():
    n, p = 4, 3
    sp_ = operators.Space(n, p, 3)
    ctrl = workloads.deformed_cube_ctrl(n, p)
    M, K = operators.free_operators(sp_, ctrl)
    x = np.random.default_rng(0).standard_normal(sp_.n_free)
    rows = np.array([0, 5, 37, sp_.n_free // 2, sp_.n_free - 1])
    np.testing.assert_allclose(operators.sampled_rows(sp_, ctrl, rows, x, "M"), (M @ x)[rows], rtol=1e-12)
    np.testing.assert_allclose(operators.sampled_rows(sp_, ctrl, rows, x, "K"), (K @ x)[rows], rtol=1e-11)
    np.testing.assert_allclose(operators.sampled_rows(sp_, ctrl, rows, x, "D"), M.diagonal()[rows], rtol=1e-13)


def test_nonpositive_jacobian_rejected():
    n, p = 2, 2
    sp_ = operators.Space(n, p, 2)
    ctrl = workloads.identity_ctrl(n, p, 2)
    ctrl[:, 0] = -ctrl[:, 0]
    with pytest.raises(ValueError):
        operators.assemble(sp_, ctrl)


def test_oracle_rows_in_worker_processes():
    # the process-pool front end of sampled_rows (used by the full-size GPU checks)
    # returns exactly the rows the oracle computes in this process
    from tests.helpers import oracle_rows, stratified_rows
    n, p = 6, 3
    ctrl = workloads.deformed_cube_ctrl(n, p)
    sp_ = operators.Space(n, p, 3)
    X = workloads.grf(n, p, seed=4)
    rows = stratified_rows((n + 1,) * 3, p, [4], [2, 4], 40, 3)
    got = oracle_rows(n, p, ctrl, {"x": X}, [("x", "M", rows), ("x", "K", rows), ("x", "D", rows)],
                      workers=2)
    for g, which in zip(got, "MKD"):
        assert np.array_equal(g, operators.sampled_rows(sp_, ctrl, rows, X, which))
