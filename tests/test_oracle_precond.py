"""Pins of the oracle's Kronecker mass preconditioner (Sec. 5.4) and solvers."""
import numpy as np
import pytest

from oracle import operators, precond, solvers
from paper_2102_11536_amd import workloads
from tests.golden.tables import pcg_tables


def _setup(dim, n, p, geometry="deformed"):
    sp_ = operators.Space(n, p, dim)
    ctrl = workloads.make_geometry(dim, n, p, geometry)
    M, K = operators.free_operators(sp_, ctrl)
    P = precond.KronPreconditioner(sp_, M.diagonal())
    return sp_, ctrl, M, K, P


@pytest.mark.parametrize("dim,n,p", [(2, 3, 2), (3, 2, 2), (3, 3, 3)])
def test_pinv_equals_dense_kron_solve(dim, n, p):
    sp_, _, M, _, P = _setup(dim, n, p)
    Pd = P.dense()
    # P is the printed product D^{1/2} Dhat^{-1/2} Mhat Dhat^{-1/2} D^{1/2}
    Mh = P.Mh[0]
    for a in range(1, dim):
        Mh = np.kron(P.Mh[a], Mh)
    Dh = np.diag(np.diag(Mh))
    D = np.diag(M.diagonal())
    Dh_mhalf = np.diag(np.diag(Dh) ** -0.5)
    Pref = np.sqrt(D) @ Dh_mhalf @ Mh @ Dh_mhalf @ np.sqrt(D)
    np.testing.assert_allclose(Pd, Pref, rtol=1e-13, atol=1e-17)
    r = np.random.default_rng(3).standard_normal(sp_.n_free)
    np.testing.assert_allclose(P.apply(r), np.linalg.solve(Pref, r), rtol=1e-9)


@pytest.mark.parametrize("dim,n,p", [(2, 4, 2), (3, 3, 3), (3, 4, 2)])
def test_identity_map_one_iteration(dim, n, p):
    # identity map: D = Dhat and M = Mhat, so P = M and PCG stops after one step
    sp_, _, M, _, P = _setup(dim, n, p, "identity")
    b = np.random.default_rng(1).standard_normal(sp_.n_free)
    x, it, ok = solvers.pcg(lambda v: M @ v, b, P.apply, tol=1e-12)
    assert ok and it == 1
    np.testing.assert_allclose(M @ x, b, rtol=1e-10, atol=1e-12)


def test_asymptotic_exactness_trend():
    # eq. limit: kappa(P^{-1/2} M P^{-1/2}) -> 1 as h -> 0 (smooth map)
    import scipy.linalg as sla
    kap = []
    for n in (3, 6, 9):
        _, _, M, _, P = _setup(3, n, 2)
        ev = sla.eigh(M.toarray(), P.dense(), eigvals_only=True)
        kap.append(ev[-1] / ev[0])
    assert kap[0] > kap[1] > kap[2] > 1.0
    assert kap[2] < 1.1


@pytest.mark.parametrize("p", [2, 3])
def test_iterations_within_paper_envelope(p):
    # Tables 1-2: single-patch means at tol 1e-12 are at most ~10 at n_sub=8
    tabs = pcg_tables()
    env = max(tabs["blade"][8][p], tabs["donut"][8][p])
    its = []
    for n in (4, 8):
        sp_, _, M, _, P = _setup(3, n, p)
        b = M @ workloads.grf(n, p, seed=5)
        x, it, ok = solvers.pcg(lambda v: M @ v, b, P.apply, tol=1e-12)
        assert ok
        its.append(it)
    assert its[1] <= its[0] <= env + 1


def test_pcg_matches_cholesky():
    sp_, _, M, _, P = _setup(3, 5, 3)
    b = np.random.default_rng(2).standard_normal(sp_.n_free)
    ch = solvers.CholeskySolver(M)
    xd = ch.solve(b)
    x, it, ok = solvers.pcg(lambda v: M @ v, b, P.apply, tol=1e-13)
    assert ok
    np.testing.assert_allclose(x, xd, rtol=1e-10, atol=1e-10 * np.max(np.abs(xd)))
    np.testing.assert_allclose(M @ xd, b, atol=1e-12 * np.max(np.abs(b)))


def test_banded_cholesky_matches_dense():
    sp_, _, M, _, _ = _setup(3, 4, 2)
    b = np.random.default_rng(4).standard_normal(sp_.n_free)
    x1 = solvers.CholeskySolver(M).solve(b)
    x2 = solvers.CholeskySolver(M, dense_limit=0).solve(b)
    np.testing.assert_allclose(x1, x2, rtol=1e-11)


def test_pcg_nonzero_guess_and_maxit():
    sp_, _, M, _, P = _setup(3, 4, 3)
    b = np.random.default_rng(5).standard_normal(sp_.n_free)
    xs = solvers.CholeskySolver(M).solve(b)
    x, it, ok = solvers.pcg(lambda v: M @ v, b, P.apply, x0=xs, tol=1e-10)
    assert ok and it == 0
    x, it, ok = solvers.pcg(lambda v: M @ v, b, P.apply, tol=1e-14, maxit=1)
    assert not ok and it == 1
