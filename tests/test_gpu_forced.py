"""Damping (Rayleigh C = cM M + cK K) and forcing in the stage equations, HIP
path against the oracle, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

from oracle import galpha
from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem

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


def _g(a, t):
    # time profile of the load and its derivatives: g(t) = cos(2 t + 0.3)
    return 2.0 ** a * np.cos(2.0 * t + 0.3 + a * np.pi / 2)


def _relM(M, a, b):
    d = a - b
    return np.sqrt(d @ (M @ d)) / max(np.sqrt(b @ (M @ b)), 1e-300)


@pytest.mark.parametrize("k,prec,cM,cK,forced", [
    (1, ga.GA_FP64, 0.8, 2e-4, True), (2, ga.GA_FP64, 0.8, 2e-4, True), (3, ga.GA_FP64, 0.5, 1e-4, True),
    (2, ga.GA_FP64, 0.0, 0.0, True), (2, ga.GA_FP64, 1.5, 0.0, False), (2, ga.GA_FP64, 0.0, 3e-4, False),
    (2, ga.GA_FP32, 0.8, 2e-4, True)])
def test_damped_forced_step_matches_oracle(k, prec, cM, cK, forced):
    _say("damped/forced", k, prec, cM, cK, forced)
    n, p = 5, 3
    pr = OracleProblem(3, n, p, geometry="deformed")
    tau = pr.tau()
    U0 = workloads.grf(n, p, seed=5)
    V0 = 0.3 * workloads.grf(n, p, seed=6)
    fvec = np.random.default_rng(7).standard_normal(pr.M.shape[0])
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
    integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12, prec=prec)
    ga.ga_integrator_set_damping(integ, cM, cK)
    state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    F0 = [_t(_g(a, 0.0) * fvec) for a in range(3 * k - 2)] if forced else None
    ga.ga_init_state_forced(integ, _t(U0), _t(V0), F0, state)
    C = (lambda y: cM * (pr.M @ y) + cK * (pr.K @ y)) if (cM or cK) else None
    Fo = (lambda a, t: _g(a, t) * fvec) if forced else None
    L = galpha.initial_state(U0, V0, k, lambda y: pr.K @ y, pr.chol.solve, apply_C=C, forcing=Fo)
    t = 0.0
    for step in range(8):
        if forced:
            ts = ga.ga_stage_times(integ, t)
            assert np.allclose(ts, galpha.stage_times(t, tau, k, 0.5))
            ga.ga_step_forced(integ, state, [_t(_g(3 * j, ts[j]) * fvec) for j in range(k)])
        else:
            ga.ga_step(integ, state, 1)
        L = galpha.step(L, tau, k, 0.5, lambda y: pr.K @ y, pr.chol.solve, apply_C=C, forcing=Fo, t=t)
        t += tau
    for s in range(3 * k):
        e = _relM(pr.M, _np(state[s]), L[s - 2])
        assert e < 1e-10, (s - 2, e)


def test_damping_argument_errors():
    pt = ga.ga_setup_patch(3, 4, 2, workloads.deformed_cube_ctrl(4, 2))
    integ = ga.ga_integrator_create(pt, 2, 0.5, 1e-3)
    for bad in ((-1.0, 0.0), (0.0, -1e-3), (float("nan"), 0.0)):
        with pytest.raises(ga.GAError):
            ga.ga_integrator_set_damping(integ, *bad)
