"""Device-side PCG control (ga_patch_set_cg): gated launches with iterations
enqueued ahead of the host's convergence read must give the iterates and the
iteration counts of the host-controlled PCG, whether the schedule guesses the
iteration counts right, too low or too high."""
import sys

import numpy as np
import pytest
import torch

from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem, rel

pytestmark = pytest.mark.gpu
# Host- and device-controlled PCG run the same kernels; their results differ only
# by the order of the FP64 atomic additions of the operator kernels (a different
# order on every run), rounding the CG recurrence amplifies over its iterations:
# up to ~1.2e-12 relative has been seen, so the bar is 1e-11, still 10x below the
# loosest tolerance the comparisons are checked at against Cholesky (1e-10)
ATOMIC_ORDER_BAR = 1e-11
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


def _solve(pt, B, rtol):
    nr = B.shape[0]
    x = torch.zeros(B.size, dtype=torch.float64, device=DEV)
    its, relres, _ = ga.ga_mass_solve(pt, _t(B.ravel()), x, nrhs=nr, rtol=rtol)
    return _np(x).reshape(nr, -1), its, relres


@pytest.mark.parametrize("n,p", [(6, 3), ((7, 5, 6), 2), (5, 4)])
def test_device_control_matches_host_and_cholesky(n, p):
    _say("cg control", n, p)
    pr = OracleProblem(3, n, p, seed=21)
    host = ga.ga_setup_patch(3, n, p, pr.ctrl)
    dev = ga.ga_setup_patch(3, n, p, pr.ctrl)
    ga.ga_patch_set_cg(host, ga.GA_CG_HOST)
    ga.ga_patch_set_cg(dev, ga.GA_CG_DEVICE)
    rng = np.random.default_rng(5)
    # a sequence whose iteration counts change: loose then tight tolerance (the
    # schedule guesses too few), tight then loose (too many), and right-hand
    # sides of different difficulty in one solve (some converge earlier)
    smooth = pr.M @ workloads.grf(n, p, seed=3)
    seq = [(rng.standard_normal((2, host.n_free)), 1e-3),
           (rng.standard_normal((2, host.n_free)), 1e-12),
           (rng.standard_normal((2, host.n_free)), 1e-12),
           (rng.standard_normal((2, host.n_free)), 1e-4),
           (np.stack([smooth, rng.standard_normal(host.n_free), smooth]), 1e-12),
           (np.stack([rng.standard_normal(host.n_free), smooth, smooth]), 1e-12),
           (np.stack([smooth, smooth, rng.standard_normal(host.n_free)]), 1e-10)]
    for i, (B, rtol) in enumerate(seq):
        xh, ih, rh = _solve(host, B, rtol)
        xd, idv, rd = _solve(dev, B, rtol)
        _say("  solve", i, "rtol", rtol, "host its", ih, "device its", idv)
        assert ih == idv, (i, ih, idv)
        for r in range(B.shape[0]):
            # the same launches up to the order of the atomic additions
            assert rel(xd[r], xh[r]) < ATOMIC_ORDER_BAR, (i, r)
            assert rd[r] <= rtol
            if rtol <= 1e-10:
                assert rel(xd[r], pr.chol.solve(B[r])) < 1e-8
    spec, checks = ga.ga_cg_stats(dev)
    _, checks_host = ga.ga_cg_stats(host)
    _say("  iterations enqueued ahead", spec, "host reads", checks, "vs", checks_host)
    assert spec > 0 and checks < checks_host


@pytest.mark.parametrize("k", [1, 2, 3])
def test_device_control_steps_match_oracle(k):
    n, p = 5, 3
    _say("cg control steps", k)
    pr = OracleProblem(3, n, p, seed=44)
    tau = pr.tau()
    U0 = workloads.grf(n, p, seed=3)
    ora = pr.run(U0, 0 * U0, k, 0.5, tau, 8)
    res = {}
    for mode in (ga.GA_CG_HOST, ga.GA_CG_DEVICE):
        pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
        ga.ga_patch_set_cg(pt, mode)
        integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12)
        state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        ga.ga_init_state(integ, _t(U0), _t(0 * U0), state)
        its = ga.ga_step(integ, state, 8)
        res[mode] = ([_np(s) for s in state], its, ga.ga_cg_stats(pt))
    assert np.array_equal(res[ga.GA_CG_HOST][1], res[ga.GA_CG_DEVICE][1])
    M = pr.M
    for s in range(3 * k):
        o = ora[8][s - 2]
        d = res[ga.GA_CG_DEVICE][0][s] - o
        assert np.sqrt(d @ (M @ d)) <= 1e-10 * max(np.sqrt(o @ (M @ o)), 1e-300), s
        assert rel(res[ga.GA_CG_DEVICE][0][s], res[ga.GA_CG_HOST][0][s]) < ATOMIC_ORDER_BAR
    _say("  host reads: host control", res[ga.GA_CG_HOST][2][1], "device control", res[ga.GA_CG_DEVICE][2][1])


def test_device_control_falls_back_with_dense_preconditioner():
    n, p = 5, 2
    pr = OracleProblem(3, n, p, seed=8)
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)      # device control is the default
    ga.ga_patch_set_pinv(pt, ga.GA_PINV_DENSE)
    B = np.random.default_rng(1).standard_normal((2, pt.n_free))
    for _ in range(2):
        x, its, _ = _solve(pt, B, 1e-12)
        for r in range(2):
            assert rel(x[r], pr.chol.solve(B[r])) < 1e-9
    assert ga.ga_cg_stats(pt)[0] == 0      # host control was used
    with pytest.raises(ga.GAError):
        ga.ga_patch_set_cg(pt, 5)


# ---- single-reduction (Chronopoulos-Gear) PCG, reductions fused into the kernels ----

@pytest.mark.parametrize("n,p", [(6, 3), ((7, 5, 6), 2), (5, 4), ((9, 4, 3), 1)])
def test_fused_single_reduction_matches_host_and_cholesky(n, p):
    # the same stopping test and, in exact arithmetic, the same iterates as the
    # classic recurrence: iteration counts within one of the host-controlled PCG
    # (a residual right at the tolerance may land on either side), solutions
    # against Cholesky, through changing schedules as in the device-control test
    _say("cg fused", n, p)
    pr = OracleProblem(3, n, p, seed=21)
    host = ga.ga_setup_patch(3, n, p, pr.ctrl)
    fus = ga.ga_setup_patch(3, n, p, pr.ctrl)
    ga.ga_patch_set_cg(host, ga.GA_CG_HOST)
    ga.ga_patch_set_cg(fus, ga.GA_CG_FUSED)
    rng = np.random.default_rng(7)
    smooth = pr.M @ workloads.grf(n, p, seed=4)
    seq = [(rng.standard_normal((2, host.n_free)), 1e-3),
           (rng.standard_normal((2, host.n_free)), 1e-12),
           (rng.standard_normal((1, host.n_free)), 1e-12),
           (rng.standard_normal((2, host.n_free)), 1e-4),
           (np.stack([smooth, rng.standard_normal(host.n_free), smooth]), 1e-12),
           (np.stack([smooth, smooth, rng.standard_normal(host.n_free), smooth]), 1e-10)]
    for i, (B, rtol) in enumerate(seq):
        xh, ih, rh = _solve(host, B, rtol)
        xf, itf, rf = _solve(fus, B, rtol)
        _say("  solve", i, "rtol", rtol, "host its", ih, "fused its", itf, "relres", rf)
        assert max(abs(a - b) for a, b in zip(ih, itf)) <= 1, (i, ih, itf)
        for r in range(B.shape[0]):
            assert rf[r] <= rtol
            if rtol <= 1e-10:
                assert rel(xf[r], pr.chol.solve(B[r])) < 1e-9
                assert rel(xf[r], xh[r]) < 1e-9
    spec, checks = ga.ga_cg_stats(fus)
    assert spec > 0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_fused_single_reduction_steps_match_oracle(k):
    n, p = 5, 3
    _say("cg fused steps", k)
    pr = OracleProblem(3, n, p, seed=44)
    tau = pr.tau()
    U0 = workloads.grf(n, p, seed=3)
    ora = pr.run(U0, 0 * U0, k, 0.5, tau, 8)
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
    ga.ga_patch_set_cg(pt, ga.GA_CG_FUSED)
    integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12)
    state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_init_state(integ, _t(U0), _t(0 * U0), state)
    ga.ga_step(integ, state, 8)
    M = pr.M
    for s in range(3 * k):
        o = ora[8][s - 2]
        d = _np(state[s]) - o
        assert np.sqrt(d @ (M @ d)) <= 1e-10 * max(np.sqrt(o @ (M @ o)), 1e-300), s


def test_fused_single_reduction_degenerate():
    # zero right-hand sides converge in zero iterations; a guess worse than zero
    # falls back; the solution of a guessed solve equals Cholesky
    pr = OracleProblem(3, 5, 3, seed=2)
    pt = ga.ga_setup_patch(3, 5, 3, pr.ctrl)
    ga.ga_patch_set_cg(pt, ga.GA_CG_FUSED)
    B = np.stack([np.zeros(pt.n_free), np.random.default_rng(3).standard_normal(pt.n_free)])
    for _ in range(2):
        x = torch.full((2 * pt.n_free,), 7.0, dtype=torch.float64, device=DEV)
        its, relres, _ = ga.ga_mass_solve(pt, _t(B.ravel()), x, nrhs=2, rtol=1e-12)
        got = _np(x).reshape(2, -1)
        assert its[0] == 0 and np.all(got[0] == 0.0), its
        assert rel(got[1], pr.chol.solve(B[1])) < 1e-10


@pytest.mark.parametrize("n,p", [(16, 2), ((11, 7), 3)])
def test_device_control_2d(n, p):
    # 2-D patches: gated 2-D operator launches and banded preconditioner passes; the
    # same iteration counts and solutions as host control, fewer host reads
    _say("cg control 2-D", n, p)
    pr = OracleProblem(2, n, p, seed=6)
    host = ga.ga_setup_patch(2, n, p, pr.ctrl)
    dev = ga.ga_setup_patch(2, n, p, pr.ctrl)
    ga.ga_patch_set_cg(host, ga.GA_CG_HOST)
    ga.ga_patch_set_cg(dev, ga.GA_CG_DEVICE)
    rng = np.random.default_rng(9)
    for i, rtol in enumerate([1e-12, 1e-12, 1e-6, 1e-12]):
        B = rng.standard_normal((2, host.n_free))
        xh, ih, _ = _solve(host, B, rtol)
        xd, idv, rd = _solve(dev, B, rtol)
        assert ih == idv, (i, ih, idv)
        for r in range(2):
            assert rel(xd[r], xh[r]) < ATOMIC_ORDER_BAR
            assert rd[r] <= rtol
            if rtol <= 1e-10:
                assert rel(xd[r], pr.chol.solve(B[r])) < 1e-9
    spec, checks = ga.ga_cg_stats(dev)
    assert spec > 0 and checks < ga.ga_cg_stats(host)[1]
