"""Glued multi-patch domain and patches with free faces: HIP path against the
oracle through the C ABI."""
import sys

import numpy as np
import pytest
import torch

from oracle import galpha, multipatch as mp, operators, precond, solvers
from paper_2102_11536_amd import ga, workloads
from tests.helpers import rel

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


@pytest.mark.parametrize("mask,n,p", [(0b111101, 4, 3), (0b001110, (5, 4, 3), 2), (0, 3, 4), (0b101010, 4, 2)])
def test_free_face_patch_matches_oracle(mask, n, p):
    _say("free faces", bin(mask), n, p)
    ctrl = workloads.deformed_cube_ctrl(n, p)
    sp_ = operators.Space(n, p, 3, dirichlet_faces=mask)
    M, K = operators.free_operators(sp_, ctrl)
    P = precond.KronPreconditioner(sp_, M.diagonal())
    pt = ga.ga_setup_patch_ex(3, n, p, ctrl, mask)
    assert pt.n_free == M.shape[0] and pt.mf == sp_.mf
    X = np.random.default_rng(2).standard_normal(pt.n_free)
    x, y = _t(X), torch.zeros(pt.n_free, dtype=torch.float64, device=DEV)
    for which, A in (("M", M), ("K", K)):
        y.zero_()
        ga.ga_apply_MK(pt, which, x, y)
        assert rel(_np(y), A @ X) < 1e-13, which
    for mode in (ga.GA_PINV_AUTO, ga.GA_PINV_DENSE):
        ga.ga_patch_set_pinv(pt, mode)
        ga.ga_apply_Pinv(pt, x, y)
        assert rel(_np(y), P.apply(X)) < 1e-12, mode


LAYOUTS = [((2, 1, 1), 4, 2), ((2, 2, 1), 3, 3), ((1, 2, 2), 3, 4), ((3, 1, 1), 3, 2)]


def _setup(P, n, p, k=2, tau=1e-3, rtol=1e-12):
    R = P[0] * P[1] * P[2]
    ctrls = [workloads.brick_ctrl(P, n, p, r) for r in range(R)]
    dom = ga.ga_mp_create(P, n, p, ctrls, k, 0.5, tau, rtol=rtol)
    gp = mp.GluedProblem(mp.Brick(P, n, p), ctrls)
    return dom, gp


@pytest.mark.parametrize("P,n,p", LAYOUTS)
def test_glued_operators_match_oracle(P, n, p):
    _say("glued ops", P, n, p)
    dom, gp = _setup(P, n, p)
    assert dom.n_global == gp.brick.n_global
    X = np.random.default_rng(3).standard_normal((2, dom.n_global))
    x = _t(X.ravel())
    y = torch.zeros_like(x)
    for which, A in (("M", gp.M), ("K", gp.K)):
        ga.ga_mp_apply(dom, which, x, y, nrhs=2)
        got = _np(y).reshape(2, -1)
        for j in range(2):
            assert rel(got[j], A @ X[j]) < 1e-13, which
    ga.ga_mp_apply(dom, "P", x, y, nrhs=2)
    got = _np(y).reshape(2, -1)
    for j in range(2):
        assert rel(got[j], gp.asm_apply(X[j])) < 1e-12


@pytest.mark.parametrize("P,n,p", LAYOUTS[:2])
def test_glued_mass_solve_matches_cholesky(P, n, p):
    dom, gp = _setup(P, n, p)
    B = np.random.default_rng(4).standard_normal(dom.n_global)
    x = torch.zeros(dom.n_global, dtype=torch.float64, device=DEV)
    its = ga.ga_mp_mass_solve(dom, _t(B), x)
    ref = solvers.CholeskySolver(gp.M).solve(B)
    _say("  P_ad iterations", its)
    assert rel(_np(x), ref) < 1e-10


@pytest.mark.parametrize("P,n,p,k", [((2, 1, 1), 4, 2, 2), ((2, 2, 1), 3, 3, 1), ((1, 1, 2), 3, 3, 3)])
def test_glued_steps_match_oracle(P, n, p, k):
    _say("glued steps", P, n, p, k)
    ctrls = [workloads.brick_ctrl(P, n, p, r) for r in range(P[0] * P[1] * P[2])]
    gp = mp.GluedProblem(mp.Brick(P, n, p), ctrls)
    import scipy.linalg as sla
    lam = float(sla.eigh(gp.K.toarray(), gp.M.toarray(), eigvals_only=True)[-1])
    tau = 0.5 * np.sqrt(ga.ga_stability_limit(0.5) / lam)
    dom = ga.ga_mp_create(P, n, p, ctrls, k, 0.5, tau, rtol=1e-12)
    U0 = workloads.brick_grf(P, n, p, seed=9)
    state = [torch.zeros(dom.n_global, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    U = _t(U0)
    ga.ga_mp_init_state(dom, U, torch.zeros_like(U), state)
    its = ga.ga_mp_step(dom, state, 6)
    ch = solvers.CholeskySolver(gp.M)
    L = galpha.initial_state(U0, 0 * U0, k, lambda y: gp.K @ y, ch.solve)
    for _ in range(6):
        L = galpha.step(L, tau, k, 0.5, lambda y: gp.K @ y, ch.solve)
    M = gp.M
    for s in range(3 * k):
        d = _np(state[s]) - L[s - 2]
        e = np.sqrt(d @ (M @ d)) / max(np.sqrt(L[s - 2] @ (M @ L[s - 2])), 1e-300)
        assert e < 1e-10, (s - 2, e)
    _say("  iterations", its.mean())


def test_glued_solve_iterations_read_ahead():
    # the iterations enqueued before the first flag read (as many as the last
    # solve needed, less one) must leave converged systems untouched: a solve
    # after a harder one, with one zero right-hand side, gives the Cholesky
    # solution, zero iterations for the zero system and the counts of a fresh solve
    P, n, p = (2, 1, 1), 4, 3
    dom, gp = _setup(P, n, p)
    rng = np.random.default_rng(8)
    ch = solvers.CholeskySolver(gp.M)
    B1 = rng.standard_normal((2, dom.n_global))
    x = torch.zeros(2 * dom.n_global, dtype=torch.float64, device=DEV)
    its1 = ga.ga_mp_mass_solve(dom, _t(B1.ravel()), x, nrhs=2)
    B2 = np.stack([rng.standard_normal(dom.n_global), np.zeros(dom.n_global)])
    its2 = ga.ga_mp_mass_solve(dom, _t(B2.ravel()), x, nrhs=2)
    got = _np(x).reshape(2, -1)
    assert rel(got[0], ch.solve(B2[0])) < 1e-10 and np.all(got[1] == 0.0)
    assert its2[1] == 0 and its2[0] > 0
    fresh, _ = _setup(P, n, p)
    x2 = torch.zeros_like(x)
    its3 = ga.ga_mp_mass_solve(fresh, _t(B2.ravel()), x2, nrhs=2)
    assert list(its2) == list(its3), (its1, its2, its3)
    # same launches; only the run-to-run order of the FP64 atomic additions differs
    assert rel(_np(x2), _np(x)) < 1e-11


def test_mp_errors():
    with pytest.raises(ga.GAError):
        ga.ga_mp_create((2, 1, 1), 3, 1, [workloads.brick_ctrl((2, 1, 1), 3, 1, r) for r in range(2)],
                        2, 0.5, 1e-3)   # p = 1 not supported by the batched kernels
    with pytest.raises(ga.GAError):
        ga.ga_setup_patch_ex(2, 4, 2, workloads.identity_ctrl(4, 2, 2), 0b0101)
