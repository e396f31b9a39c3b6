"""Batched 1-D wave problems (ga_wave1d_*, the dispersion study of Sec. 6.2) and
the two-parameter family rho_s <= rho_b, through the C ABI, against the oracle."""
import sys

import numpy as np
import pytest
import torch

from oracle import dispersion, galpha
from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ga.load_library()


@pytest.mark.parametrize("N,p", [(13, 2), (9, 3), (20, 4), (1, 4), (3, 1)])
def test_operators_load_and_solve_match_oracle(N, p):
    _say("wave1d operators", N, p)
    ora = dispersion.Wave1D(N, p)
    js = np.array([1.0, 2.0, 5.0])
    w = ga.Wave1D(N, p, 1.0 / js ** 2, 1, 0.5, 0.5, 1e-3)
    assert w.m == ora.n_free
    X = np.random.default_rng(2).standard_normal((3, w.m))
    x, y = _t(X.ravel()), torch.empty(3 * w.m, dtype=torch.float64, device=DEV)
    for which, A in (("M", ora.M), ("K", ora.K)):
        ga.ga_wave1d_apply(w, which, x, y)
        got = _np(y).reshape(3, -1)
        for r in range(3):
            assert rel(got[r], A @ X[r]) < 1e-13, which
    ga.ga_wave1d_apply(w, "S", x, y)
    got = _np(y).reshape(3, -1)
    for r in range(3):
        assert rel(got[r], ora.chol.solve(X[r])) < 1e-11
    f = torch.empty_like(y)
    ga.ga_wave1d_load_sine(w, js, f)
    got = _np(f).reshape(3, -1)
    for r, j in enumerate(js):
        assert rel(got[r], ora.load(j)) < 1e-13


@pytest.mark.parametrize("k,rb,rs", [(1, 0.5, 0.5), (2, 0.5, 0.5), (2, 0.8, 0.3), (3, 0.9, 0.0)])
def test_steps_match_oracle(k, rb, rs):
    N, p, nsteps = 20, 4, 40
    _say("wave1d steps", k, rb, rs)
    ora = dispersion.Wave1D(N, p)
    lam = ora.discrete_eigenvalues()[-1]
    js = np.array([3.0, 4.0, 7.0, 11.0])
    tau = 0.9 * np.sqrt(ga.ga_stability_limit2(rb, rs) / lam) * js[0]   # stable for every system
    w = ga.Wave1D(N, p, 1.0 / js ** 2, k, rb, rs, tau)
    f = torch.empty(w.n_total, dtype=torch.float64, device=DEV)
    ga.ga_wave1d_load_sine(w, js, f)
    U0 = torch.empty_like(f)
    ga.ga_wave1d_apply(w, "S", f, U0)
    state = [torch.zeros_like(f) for _ in range(3 * k)]
    ga.ga_wave1d_init_state(w, U0, torch.zeros_like(U0), state)
    ga.ga_wave1d_step(w, state, nsteps)
    got = [_np(s).reshape(len(js), -1) for s in state]
    M = ora.M
    for r, j in enumerate(js):
        w2 = 1.0 / j ** 2
        apply_K = lambda y: w2 * (ora.K @ y)
        U = ora.projection(j)
        L = galpha.initial_state(U, 0 * U, k, apply_K, ora.chol.solve)
        for _ in range(nsteps):
            L = galpha.step(L, tau, k, rb, apply_K, ora.chol.solve, rho_s=rs)
        # rounding in L^a (the a-th derivative of the acceleration) is amplified
        # relative to the solution by (highest discrete frequency / solution
        # frequency)^a: the bar is 1e-10 for U, V, A and grows by that ratio
        ratio = np.sqrt(w2 * lam) / np.pi
        for s in range(3 * k):
            a = s - 2
            d = got[s][r] - L[a]
            e = np.sqrt(d @ (M @ d)) / max(np.sqrt(L[a] @ (M @ L[a])), 1e-300)
            assert e < 1e-10 * ratio ** max(a, 0), (j, s, e)


def test_dispersion_study_small():
    # the study's shape at N = 40: stable wavenumbers at tau = 0.05, T = 5, both
    # orders; errors as the oracle's and the order-4 scheme better at low j
    N, p, tau, T = 40, 4, 0.05, 5.0
    ora = dispersion.Wave1D(N, p)
    lam = ora.discrete_eigenvalues()[-1]
    j0 = dispersion.smallest_stable_j(lam, 0.5, tau)
    js = np.arange(j0, N + 1, dtype=np.float64)
    n = int(round(T / tau))
    err = {}
    for k in (1, 2):
        w = ga.Wave1D(N, p, 1.0 / js ** 2, k, 0.5, 0.5, tau)
        f = torch.empty(w.n_total, dtype=torch.float64, device=DEV)
        ga.ga_wave1d_load_sine(w, js, f)
        U0 = torch.empty_like(f)
        ga.ga_wave1d_apply(w, "S", f, U0)
        state = [torch.zeros_like(f) for _ in range(3 * k)]
        ga.ga_wave1d_init_state(w, U0, torch.zeros_like(U0), state)
        ga.ga_wave1d_step(w, state, n)
        U = _np(state[0]).reshape(len(js), -1)
        err[k] = np.array([ora.rel_l2_error(U[r], j, T) for r, j in enumerate(js)])
        for r in (0, len(js) // 2, len(js) - 1):
            ref = ora.rel_l2_error(ora.run(js[r], k, 0.5, tau, n), js[r], T)
            assert abs(err[k][r] - ref) <= 1e-8 * max(ref, 1e-6), (k, js[r], err[k][r], ref)
    _say("  j", js[:4], "k=1", err[1][:4], "k=2", err[2][:4])
    assert np.all(err[2][:3] < err[1][:3])


def test_two_parameter_integrator_matches_oracle():
    k, n, p, rb, rs = 2, 5, 3, 0.8, 0.3
    pr = OracleProblem(3, n, p, seed=44)
    lam = float(np.max(np.abs(np.linalg.eigvals(np.linalg.solve(pr.M.toarray(), pr.K.toarray())))))
    tau = 0.5 * np.sqrt(ga.ga_stability_limit2(rb, rs) / lam)
    U0 = workloads.grf(n, p, seed=3)
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
    integ = ga.ga_integrator_create(pt, k, rb, tau, rtol=1e-12)
    ga.ga_integrator_set_rho(integ, rb, rs)
    state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_init_state(integ, _t(U0), _t(0 * U0), state)
    ga.ga_step(integ, state, 10)
    K, ch = pr.K, pr.chol
    L = galpha.initial_state(U0, 0 * U0, k, lambda y: K @ y, ch.solve)
    for _ in range(10):
        L = galpha.step(L, tau, k, rb, lambda y: K @ y, ch.solve, rho_s=rs)
    M = pr.M
    for s in range(3 * k):
        d = _np(state[s]) - L[s - 2]
        assert np.sqrt(d @ (M @ d)) <= 1e-10 * np.sqrt(L[s - 2] @ (M @ L[s - 2])), s
    for rb_, rs_ in ((0.5, 0.5), (0.8, 0.3), (0.99, 0.5)):
        assert abs(ga.ga_stability_limit2(rb_, rs_) - dispersion.stability_limit_closed(rb_, rs_)) < 1e-12


def test_errors():
    with pytest.raises(ga.GAError):
        ga.Wave1D(10, 3, [1.0], 2, 0.3, 0.5, 0.01)      # rho_s > rho_b
    with pytest.raises(ga.GAError):
        ga.Wave1D(10, 3, [0.0], 2, 0.5, 0.5, 0.01)      # omega^2 = 0
    with pytest.raises(ga.GAError):
        ga.Wave1D(10, 5, [1.0], 2, 0.5, 0.5, 0.01)      # p > 4
    pt = ga.ga_setup_patch(3, 3, 2, workloads.deformed_cube_ctrl(3, 2))
    integ = ga.ga_integrator_create(pt, 2, 0.5, 1e-3)
    with pytest.raises(ga.GAError):
        ga.ga_integrator_set_rho(integ, 0.5, 0.6)
