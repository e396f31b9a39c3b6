"""Pins of the 1-D dispersion oracle (oracle/dispersion.py, Sec. 6.2) and of the
two-parameter family rho_s <= rho_b (Remark in Sec. 3)."""
import numpy as np
import pytest

from oracle import dispersion, galpha


@pytest.fixture(scope="module")
def w40():
    return dispersion.Wave1D(40, 4)


def test_projection_converges_at_order_p_plus_1():
    # L2 projection error of sin(j pi x): O(h^{p+1}); pins the load vector, the
    # 1-D mass matrix and the quadrature of the error measure together
    for p in (2, 3, 4):
        e = [dispersion.Wave1D(N, p).rel_l2_error(dispersion.Wave1D(N, p).projection(2), 2, 0.0)
             for N in (16, 32)]
        rate = np.log2(e[0] / e[1])
        assert abs(rate - (p + 1)) < 0.25, (p, rate)


def test_exact_solution_norm_and_error_measure(w40):
    # the discrete field equal to the projection at t = 0 and its negative at t = 1
    # (cos(pi) = -1) give the same relative error; a zero field gives error 1
    U = w40.projection(3)
    assert abs(w40.rel_l2_error(U, 3, 0.0) - w40.rel_l2_error(-U, 3, 1.0)) < 1e-15
    assert abs(w40.rel_l2_error(0 * U, 3, 0.0) - 1.0) < 1e-14


def test_discrete_eigenvalues_superconverge():
    # lambda_h(j) -> (j pi)^2 with relative error O(h^{2p}) for a fixed j
    p = 3
    err = []
    for N in (10, 20):
        lam = dispersion.Wave1D(N, p).discrete_eigenvalues()
        err.append(abs(lam[1] - (2 * np.pi) ** 2) / (2 * np.pi) ** 2)
    assert abs(np.log2(err[0] / err[1]) - 2 * p) < 0.5


def test_omega_enters_as_time_rescaling(w40):
    # M U'' + omega^2 K U = 0 with step tau is the omega = 1 problem with step
    # omega tau (the scheme is homogeneous in tau): the displacements agree
    j, k, tau, n = 7, 2, 0.01, 30
    U1 = w40.run(j, k, 0.5, tau, n)
    K, ch = w40.K, w40.chol
    U0 = w40.projection(j)
    L = galpha.initial_state(U0, 0 * U0, k, lambda y: K @ y, ch.solve)
    for _ in range(n):
        L = galpha.step(L, tau / j, k, 0.5, lambda y: K @ y, ch.solve)
    assert np.linalg.norm(L[-2] - U1) <= 1e-11 * np.linalg.norm(U1)


def test_order_2k_in_time_and_small_tau_limit():
    # j = 1 on a coarse mesh (every mode stable for tau <= 0.04): halving tau
    # divides the time error at T = 0.75 (the distance to a k = 3 run with
    # tau / 16) by ~2^{2k}; at tau = 0.005 the k = 2 run is
    # at the projection error, k = 1 well above it
    w = dispersion.Wave1D(8, 4)
    j, T = 1, 0.75
    ref = w.run(j, 3, 0.5, 0.0375 / 16, 320)            # the semi-discrete solution at T
    for k, lo, hi in ((1, 3.5, 4.5), (2, 13.0, 19.0)):
        e = [np.linalg.norm(w.run(j, k, 0.5, tau, int(round(T / tau))) - ref) for tau in (0.0375, 0.01875)]
        assert lo < e[0] / e[1] < hi, (k, e)
    proj = w.rel_l2_error(w.projection(j), j, 0.0)
    e2 = w.rel_l2_error(w.run(j, 2, 0.5, 0.005, 150), j, T)
    e1 = w.rel_l2_error(w.run(j, 1, 0.5, 0.005, 150), j, T)
    assert e2 < 3 * proj < e1, (proj, e2, e1)


def test_stable_range(w40):
    # below the smallest stable j the run grows without bound, at it the run stays bounded
    lam = w40.discrete_eigenvalues()[-1]
    tau = 0.05
    j0 = dispersion.smallest_stable_j(lam, 0.5, tau)
    assert tau ** 2 * lam / j0 ** 2 <= dispersion.stability_limit_closed(0.5)
    assert tau ** 2 * lam / (j0 - 1) ** 2 > dispersion.stability_limit_closed(0.5)
    n = 100
    assert w40.rel_l2_error(w40.run(j0, 2, 0.5, tau, n), j0, n * tau) < 1.0
    assert w40.rel_l2_error(w40.run(j0 - 1, 2, 0.5, tau, n), j0 - 1, n * tau) > 1e3


# ---- the two-parameter family rho_s <= rho_b ---------------------------------

@pytest.mark.parametrize("rb,rs", [(0.5, 0.5), (0.8, 0.3), (0.9, 0.0), (0.99, 0.5), (0.3, 0.0)])
def test_two_parameter_stability_limit(rb, rs):
    # bisection on the spectral radius equals the lambda = -1 root of the type-k
    # polynomial for every k; rho_s = rho_b is the one-parameter family
    ref = dispersion.stability_limit_closed(rb, rs)
    for k in (1, 2, 3):
        assert abs(galpha.stability_limit(k, rb, rho_s=rs) - ref) < 1e-7
    if rs == rb:
        assert galpha.block_params(2, rb, rs) == galpha.block_params(2, rb)


@pytest.mark.parametrize("rb,rs", [(0.8, 0.3), (0.6, 0.2), (0.9, 0.0)])
def test_two_parameter_bifurcation_roots(rb, rs):
    # eq. root: at Theta = Omega_b the last block's eigenvalues are -rho_b (double)
    # and -rho_s
    _, _, omega_b, _ = galpha.printed_type_k(rb, rs)
    G = galpha.amplification_matrix(2, rb, omega_b, rho_s=rs)
    ev = np.sort(np.linalg.eigvals(G[3:, 3:]).real)
    np.testing.assert_allclose(ev, np.sort([-rb, -rb, -rs]), atol=1e-6)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_two_parameter_family_keeps_order_2k(k):
    # SDOF x'' = -w^2 x from exact data: error ratio ~2^{2k} when tau halves
    rb, rs, w, T = 0.8, 0.3, 2.6 * np.pi, 0.73
    errs = []
    for n in (100, 200):
        tau = T / n
        N = 3 * k - 3
        L = {-2: 1.0, -1: 0.0}
        for a in range(0, N + 1):
            L[a] = -w ** 2 * L[a - 2]
        for _ in range(n):
            L = galpha.step(L, tau, k, rb, lambda y: w ** 2 * y, lambda b: b, rho_s=rs)
        errs.append(abs(L[-2] - np.cos(w * T)))
    assert abs(np.log2(errs[0] / errs[1]) - 2 * k) < 0.35, errs


@pytest.mark.parametrize("k", [2, 3])
@pytest.mark.parametrize("rb,rs", [(0.8, 0.3), (0.6, 0.2), (0.9, 0.0), (0.5, 0.5)])
def test_two_parameter_type_j_block_roots(k, rb, rs):
    # eq. root for the blocks j < k under the sign reading: the printed type-j
    # Omega_b evaluated at (-rho_b, -rho_s) is the type-k Omega_b, and there every
    # block j < k has the eigenvalues -rho_b (double) and -rho_s.  A flipped sign
    # (type-j formulas at +rho) moves these roots off -rho_b, -rho_s.
    _, _, omega_bj, _ = galpha.printed_type_j(-rb, -rs)
    _, _, omega_bk, _ = galpha.printed_type_k(rb, rs)
    assert abs(omega_bj - omega_bk) < 1e-14
    G = galpha.amplification_matrix(k, rb, omega_bj, rho_s=rs)
    tol = 2e-4 if rb == rs else 1e-6  # a triple root is resolved to ~eps^(1/3)
    for j in range(k - 1):
        ev = np.linalg.eigvals(G[3 * j:3 * j + 3, 3 * j:3 * j + 3])
        assert np.max(np.abs(ev.imag)) < tol
        np.testing.assert_allclose(np.sort(ev.real), np.sort([-rb, -rb, -rs]), atol=tol)
    # the literal sign: the type-j block at +rho has other roots at this Theta
    a, b, _, _ = galpha.printed_type_j(rb, rs)
    th = omega_bj
    g = 0.5 - 1 + a
    blk = np.array([[a - b * th, a - b * th, 0.5 * (a - b * (th + 2))],
                    [-g * th, a - g * th, a - 0.5 * g * (th + 2)],
                    [-th, -th, a - 1 - 0.5 * th]]) / a
    ev = np.sort(np.linalg.eigvals(blk).real)
    assert np.max(np.abs(ev - np.sort([-rb, -rb, -rs]))) > 1e-2
