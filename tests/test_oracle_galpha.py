"""Pins of the oracle's order-2k integrator (Sec. 3-4) against the matrices,
polynomials and claims the paper prints, textbook Hulbert-Chung parameters and
exact solutions."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import galpha, operators, solvers
from paper_2102_11536_amd import workloads


def lam_j(al, be, ga, th):
    # printed diagonal block for j < k (eq. HOblock, also Lambda_1 of Sec. 3)
    return np.array([[al - be * th, al - be * th, 0.5 * (al - be * (th + 2))],
                     [-ga * th, al - ga * th, al - 0.5 * ga * (th + 2)],
                     [-th, -th, al - 1 - 0.5 * th]]) / al


def lam_k(al, be, ga, th):
    # printed last diagonal block (eq. HOblock, Lambda_2 of Sec. 3)
    return np.array([[al - be * th, al, 0.5 * al - be],
                     [-ga * th, al, al - ga],
                     [-th, 0.0, al - 1]]) / al


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("rho", [0.0, 0.3, 0.5, 0.8])
@pytest.mark.parametrize("theta", [0.05, 1.0, 3.0])
def test_amplification_blocks_match_printed(k, rho, theta):
    G = galpha.amplification_matrix(k, rho, theta)
    prm = galpha.block_params(k, rho)
    for j in range(k):
        al, be, ga, _ = prm[j]
        ref = lam_k(al, be, ga, theta) if j == k - 1 else lam_j(al, be, ga, theta)
        np.testing.assert_allclose(G[3 * j:3 * j + 3, 3 * j:3 * j + 3], ref, atol=1e-13)
        # block upper triangular (eq. HOampblock)
        assert np.all(G[3 * j + 3:, 3 * j:3 * j + 3] == 0)


@pytest.mark.parametrize("rho", [0.2, 0.5, 0.9])
@pytest.mark.parametrize("theta", [0.3, 2.0])
def test_characteristic_polynomials(rho, theta):
    # eq. charact, printed for Lambda_1 (type j) and Lambda_2 (type k)
    prm = galpha.block_params(2, rho)
    G = galpha.amplification_matrix(2, rho, theta)
    a1, b1, g1, _ = prm[0]
    a2, b2, g2, _ = prm[1]
    T = theta
    c1 = [2 * a1, T * (2 * b1 + 2 * g1 + 1) - 6 * a1 + 2, T * (-4 * b1 - 2 * g1 + 1) + 6 * a1 - 4,
          2 * b1 * T - 2 * a1 + 2]
    c2 = [2 * a2, 2 * T * b2 - 6 * a2 + 2, T * (-4 * b2 + 2 * g2 + 1) + 6 * a2 - 4,
          T * (2 * b2 + 1 - 2 * g2) - 2 * a2 + 2]
    for blk, c in ((G[:3, :3], c1), (G[3:, 3:], c2)):
        ref = np.poly(blk) * c[0]
        np.testing.assert_allclose(ref, c, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_low_frequency_eigenvalues(k):
    # eq. t0: as Theta -> 0 each block has eigenvalues 1, 1, 1 - 1/alpha
    rho = 0.4
    ev = np.sort_complex(np.linalg.eigvals(galpha.amplification_matrix(k, rho, 1e-12)))
    al = galpha.block_params(k, rho)[0][0]
    ref = np.sort_complex(np.array([1.0] * (2 * k) + [1 - 1 / al] * k, complex))
    np.testing.assert_allclose(ev, ref, atol=2e-5)


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.8])
def test_stability_limit_independent_of_k(rho):
    # abstract and Remark of Sec. 4: the stability region does not change with k.
    # The limit is the lambda = -1 root of the printed type-k characteristic
    # polynomial: Theta(8 beta - 4 gamma) + 8 - 16 alpha = 0.
    al, be, ga, _ = galpha.block_params(1, rho)[0]
    ref = (16 * al - 8) / (8 * be - 4 * ga)
    for k in (1, 2, 3):
        assert abs(galpha.stability_limit(k, rho) - ref) < 1e-7
    if rho == 0.0:
        assert abs(ref - 2.4) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("rho", [0.3, 0.5, 0.7])
def test_bifurcation_triple_eigenvalue(k, rho):
    # eq. root: at Theta = Omega_b all eigenvalues of every block equal -rho
    _, _, omega_b, _ = galpha.printed_type_k(rho, rho)
    ev = np.linalg.eigvals(galpha.amplification_matrix(k, rho, omega_b))
    np.testing.assert_allclose(ev, -rho, atol=2e-4)  # triple root: error ~ eps^(1/3)


def test_literal_sign_breaks_k_invariance():
    # documents the reading: the printed type-j formulas at +rho make blocks j<k
    # unstable well below the type-k limit
    a, b, _, _ = galpha.printed_type_j(0.5, 0.5)
    th = 2.0
    blk = lam_j(a, b, 0.5 - 1 + a, th)
    assert np.max(np.abs(np.linalg.eigvals(blk))) > 1.0
    assert galpha.spectral_radius(2, 0.5, th) <= 1.0 + 1e-12


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9])
def test_k1_is_hulbert_chung(rho):
    # explicit generalized-alpha of Hulbert & Chung: alpha_m = (2 rho - 1)/(1 + rho),
    # beta = (5 - 3 rho)/((1 + rho)^2 (2 - rho)), gamma = 3/2 - alpha_m; the
    # paper's alpha weights the new acceleration, i.e. alpha = 1 - alpha_m.
    al, be, ga, af = galpha.block_params(1, rho)[0]
    am = (2 * rho - 1) / (1 + rho)
    assert abs(al - (1 - am)) < 1e-14
    assert abs(be - (5 - 3 * rho) / ((1 + rho) ** 2 * (2 - rho))) < 1e-14
    assert abs(ga - (1.5 - am)) < 1e-14 and af == 0.0


def _sdof_error(k, rho, om, T, nst):
    lam = om * om
    tau = T / nst
    L = {a: om ** (a + 2) * np.cos((a + 2) * np.pi / 2) for a in range(-2, 3 * k - 2)}
    for _ in range(nst):
        L = galpha.step(L, tau, k, rho, lambda y: lam * y, lambda b: b)
    return abs(L[-2] - np.cos(om * T))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_sdof_order_2k(k):
    # Theorem 2: order 2k in time, checked against x(t) = cos(omega t)
    # a generic end time (at omega T = 2 pi the leading phase error vanishes)
    om, T = 2.6 * np.pi, 0.73
    ns = (100, 200, 400) if k < 3 else (40, 80, 160)
    e = [_sdof_error(k, 0.5, om, T, n) for n in ns]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    assert all(abs(r - 2 * k) < 0.25 for r in rates), rates


def _wave2d(n, p):
    sp_ = operators.Space(n, p, 2)
    ctrl = workloads.identity_ctrl(n, p, 2)
    M, K = operators.free_operators(sp_, ctrl)
    return sp_, M.toarray(), K.toarray()


@pytest.mark.parametrize("k", [1, 2])
def test_eigenvector_data_reduces_to_sdof(k):
    # with U0 an eigenvector of (K, M) the PDE run is the scalar run times it
    n, p, rho = 6, 2, 0.5
    _, M, K = _wave2d(n, p)
    lam, V = sla.eigh(K, M)
    v = V[:, 3]
    tau = 0.02
    ch = solvers.CholeskySolver(M)
    L = galpha.initial_state(v, 0 * v, k, lambda y: K @ y, ch.solve)
    s = galpha.initial_state(1.0, 0.0, k, lambda y: lam[3] * y, lambda b: b)
    for _ in range(25):
        L = galpha.step(L, tau, k, rho, lambda y: K @ y, ch.solve)
        s = galpha.step(s, tau, k, rho, lambda y: lam[3] * y, lambda b: b)
    for a in L:
        np.testing.assert_allclose(L[a], s[a] * v, atol=1e-9 * max(1, abs(s[a])))


def test_standing_wave_2d():
    # closed form u = sin(pi x) sin(pi y) cos(sqrt(2) pi t) (unit square, omega = 1):
    # time error against the semi-discrete solution falls at order 2k, and the
    # full error against the closed form sits at the spatial floor.
    n, p, rho = 16, 2, 0.5
    sp_, M, K = _wave2d(n, p)
    # L2 projection of u0 (load vector by the same quadrature)
    from oracle import bspline
    xq, wq, Bx, _ = bspline.tables_1d(n, p)
    f1 = np.sin(np.pi * xq) * wq
    b1 = (Bx.T @ f1)[1:-1]
    U0 = np.linalg.solve(M, np.kron(b1, b1))
    lam, V = sla.eigh(K, M)
    c0 = V.T @ M @ U0
    T = 0.5
    ch = solvers.CholeskySolver(M)

    def run(k, nst):
        tau = T / nst
        L = galpha.initial_state(U0, 0 * U0, k, lambda y: K @ y, ch.solve)
        for _ in range(nst):
            L = galpha.step(L, tau, k, rho, lambda y: K @ y, ch.solve)
        return L[-2]

    exact = V @ (c0 * np.cos(np.sqrt(lam) * T))
    for k, ns in ((1, (200, 400, 800)), (2, (100, 200, 400))):
        errs = [np.sqrt((run(k, nn) - exact) @ M @ (run(k, nn) - exact)) for nn in ns]
        rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(abs(r - 2 * k) < 0.3 for r in rates), (k, rates, errs)
    # closed form at T: coefficients of the L2 projection of u(T)
    Uex = U0 * np.cos(np.sqrt(2) * np.pi * T)
    d = run(2, 400) - Uex
    assert np.sqrt(d @ M @ d) < 1e-6


# ---- damping and forcing (stage equations ho1 with C and F) ----------------

def _damped_forced_exact(lam, c, A, Om, x0, v0, t):
    """x'' + c x' + lam x = A sin(Om t), x(0) = x0, x'(0) = v0 (underdamped)."""
    D = (lam - Om ** 2) ** 2 + (c * Om) ** 2
    a, b = A * (lam - Om ** 2) / D, -A * c * Om / D
    wd = np.sqrt(lam - c * c / 4)
    C1 = x0 - b
    C2 = (v0 - a * Om + 0.5 * c * C1) / wd
    return a * np.sin(Om * t) + b * np.cos(Om * t) + np.exp(-0.5 * c * t) * (C1 * np.cos(wd * t) + C2 * np.sin(wd * t))


def _damped_forced_error(k, nst, c=1.3, A=5.0, damping_args=None):
    lam, Om, T, x0, v0, rho = (2.6 * np.pi) ** 2, 3.1, 0.73, 1.0, -0.4, 0.5
    tau = T / nst
    F = (lambda a, t: A * Om ** a * np.sin(Om * t + a * np.pi / 2)) if A else None
    L = galpha.initial_state(x0, v0, k, lambda y: lam * y, lambda b: b, apply_C=lambda y: c * y, forcing=F)
    t = 0.0
    for _ in range(nst):
        L = galpha.step(L, tau, k, rho, lambda y: lam * y, lambda b: b, apply_C=lambda y: c * y,
                        forcing=F, t=t)
        t += tau
    return abs(L[-2] - _damped_forced_exact(lam, c, A, Om, x0, v0, T))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_damped_forced_sdof_order_2k(k):
    # order 2k against the closed-form damped, forced oscillator; k = 3 is
    # still slightly pre-asymptotic (rates approach 6 from above)
    ns = (200, 400, 800) if k < 3 else (80, 160, 320)
    e = [_damped_forced_error(k, n) for n in ns]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
    assert all(2 * k - 0.35 < r < 2 * k + 0.9 for r in rates), rates
    assert rates[-1] <= rates[0] + 0.3 or k < 3


def test_literal_damping_argument_is_first_order(monkeypatch):
    # C acting on L^{a_j-1}_n (the printed stage equations) instead of the
    # predictor drops the scheme to first order: the reading is what the pin fixes
    monkeypatch.setattr(galpha, "damping_arguments",
                        lambda L, T, k: [L[3 * j - 4] for j in range(1, k + 1)])
    e = [_damped_forced_error(2, n, A=0.0) for n in (200, 400)]
    assert abs(np.log2(e[0] / e[1]) - 1.0) < 0.2


@pytest.mark.parametrize("k", [1, 2, 3])
def test_rayleigh_damped_forced_pde_reduces_to_sdof(k):
    # U0 an eigenvector v of (K, M), C = cM M + cK K, F = g(t) M v: the PDE run is
    # the scalar run with c = cM + cK lambda and force g(t), times v
    n, p, rho, cM, cK = 6, 2, 0.5, 0.7, 2e-3
    _, M, K = _wave2d(n, p)
    lam, V = sla.eigh(K, M)
    v, l3 = V[:, 3], lam[3]
    Mv = M @ v
    g = lambda a, t: 3.0 * 2.0 ** a * np.cos(2.0 * t + a * np.pi / 2)
    tau = 0.02
    ch = solvers.CholeskySolver(M)
    C = lambda y: cM * (M @ y) + cK * (K @ y)
    L = galpha.initial_state(v, 0.5 * v, k, lambda y: K @ y, ch.solve, apply_C=C,
                             forcing=lambda a, t: g(a, t) * Mv)
    s = galpha.initial_state(1.0, 0.5, k, lambda y: l3 * y, lambda b: b,
                             apply_C=lambda y: (cM + cK * l3) * y, forcing=g)
    t = 0.0
    for _ in range(25):
        L = galpha.step(L, tau, k, rho, lambda y: K @ y, ch.solve, apply_C=C,
                        forcing=lambda a, tt: g(a, tt) * Mv, t=t)
        s = galpha.step(s, tau, k, rho, lambda y: l3 * y, lambda b: b,
                        apply_C=lambda y: (cM + cK * l3) * y, forcing=g, t=t)
        t += tau
    for a in range(-2, 3 * k - 2):
        assert np.allclose(L[a], s[a] * v, rtol=1e-9, atol=1e-9 * np.abs(s[a]) + 1e-12)


def test_no_damping_no_forcing_is_the_plain_step():
    rng = np.random.default_rng(0)
    L = {a: rng.standard_normal(5) for a in range(-2, 4)}
    A = np.diag(rng.uniform(1, 2, 5))
    a1 = galpha.step(L, 0.01, 2, 0.5, lambda y: A @ y, lambda b: b)
    a2 = galpha.step(L, 0.01, 2, 0.5, lambda y: A @ y, lambda b: b, apply_C=lambda y: 0 * y,
                     forcing=lambda a, t: np.zeros(5), t=3.0)
    for a in a1:
        assert np.array_equal(a1[a], a2[a])
