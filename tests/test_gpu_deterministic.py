"""Deterministic mode (ga_patch_set_deterministic): operator applies, solves and steps
are bitwise reproducible, equal the oracle to the usual bars, and host- and
device-controlled PCG give bitwise the same iterates in this mode (the default mode
differs from run to run in the last bits through the order of the FP64 atomic
additions of shared coefficients)."""
import sys

import numpy as np
import pytest
import torch

from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem, rel

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ga.load_library()


# several xy tiles per axis and (with 4 layers per workgroup) several z ranges, so
# every colour class is populated; p = 4 takes the 3-element tiles (9 classes in x-y)
CASES = [((9, 7, 10), 3, 4), ((8, 10, 9), 2, 4), ((7, 6, 9), 4, 4), ((9, 9, 6), 3, 0)]


@pytest.mark.parametrize("n,p,ze", CASES)
def test_deterministic_applies_bitwise_and_match_oracle(n, p, ze):
    _say("deterministic apply", n, p, ze)
    pr = OracleProblem(3, n, p, seed=13)
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
    ga.ga_patch_set_layers(pt, ze, ze)
    ga.ga_patch_set_deterministic(pt, True)
    X = np.random.default_rng(2).standard_normal((3, pt.n_free))
    x = _t(X.ravel())
    for which, A in (("M", pr.M), ("K", pr.K)):
        for nrhs in (1, 2, 3):
            y1 = torch.empty(nrhs * pt.n_free, dtype=torch.float64, device=DEV)
            y2 = torch.empty_like(y1)
            ga.ga_apply_MK(pt, which, x, y1, nrhs=nrhs)
            ga.ga_apply_MK(pt, which, x, y2, nrhs=nrhs)
            torch.cuda.synchronize()
            assert torch.equal(y1, y2), (which, nrhs)
            got = y1.cpu().numpy().reshape(nrhs, -1)
            for r in range(nrhs):
                assert rel(got[r], A @ X[r]) < 1e-13, (which, nrhs, r)


def test_deterministic_solves_and_steps_bitwise():
    n, p, k = (9, 7, 10), 3, 2
    pr = OracleProblem(3, n, p, seed=44)
    tau = pr.tau()
    U0 = workloads.grf(n, p, seed=3)
    B = np.random.default_rng(5).standard_normal((2, pr.M.shape[0]))
    outs = {}
    for mode in (ga.GA_CG_HOST, ga.GA_CG_DEVICE, ga.GA_CG_DEVICE):
        pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
        ga.ga_patch_set_layers(pt, 4, 4)
        ga.ga_patch_set_deterministic(pt, True)
        ga.ga_patch_set_cg(pt, mode)
        for _ in range(2):   # the second solve runs on the first one's schedule (device control)
            x = torch.zeros(2 * pt.n_free, dtype=torch.float64, device=DEV)
            its, _, _ = ga.ga_mass_solve(pt, _t(B.ravel()), x, nrhs=2, rtol=1e-12)
        integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12)
        st = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        u = _t(U0)
        ga.ga_init_state(integ, u, torch.zeros_like(u), st)
        ga.ga_step(integ, st, 6)
        torch.cuda.synchronize()
        outs.setdefault(mode, []).append((x.clone(), its, [s.clone() for s in st]))
    (xh, ih, sh), = outs[ga.GA_CG_HOST]
    (xd1, id1, sd1), (xd2, id2, sd2) = outs[ga.GA_CG_DEVICE]
    assert ga.ga_cg_stats(pt)[0] > 0   # the last patch enqueued iterations ahead
    # run to run, and host against device control: the same kernels in the same order
    assert torch.equal(xd1, xd2) and torch.equal(xh, xd1)
    assert ih == id1 == id2
    for a, b, c in zip(sh, sd1, sd2):
        assert torch.equal(b, c) and torch.equal(a, b)
    got = xh.cpu().numpy().reshape(2, -1)
    for r in range(2):
        assert rel(got[r], pr.chol.solve(B[r])) < 1e-10
    ora = pr.run(U0, 0 * U0, k, 0.5, tau, 6)[-1]
    M = pr.M
    for s in range(3 * k):
        d = sh[s].cpu().numpy() - ora[s - 2]
        assert np.sqrt(d @ (M @ d)) <= 1e-10 * max(np.sqrt(ora[s - 2] @ (M @ ora[s - 2])), 1e-300)


@pytest.mark.parametrize("guess", [ga.GA_GUESS_ZERO, ga.GA_GUESS_EXTRAP])
def test_checkpoint_resume_is_bitwise(guess):
    # checkpoint after 5 of 9 steps (state vectors and the ring of past stage solutions
    # copied to host memory), resume in a fresh integrator: the last 4 steps are
    # bitwise those of the uninterrupted run (deterministic mode, FP64 solves)
    _say("checkpoint/resume", guess)
    n, p, k = (7, 6, 5), 3, 2
    pr = OracleProblem(3, n, p, seed=12)
    pt = ga.ga_setup_patch(3, n, p, pr.ctrl)
    ga.ga_patch_set_deterministic(pt, 1)
    tau = pr.tau()
    U0 = _t(workloads.grf(n, p, seed=6))
    nf = pt.n_free

    def fresh():
        return ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-10, guess=guess)

    def started():
        integ = fresh()
        st = [torch.zeros(nf, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        ga.ga_init_state(integ, U0, torch.zeros_like(U0), st)
        return integ, st

    integ, st = started()
    ga.ga_step(integ, st, 9)
    ref = [s_.cpu().numpy() for s_ in st]
    integ.close()

    integ, st = started()
    ga.ga_step(integ, st, 5)
    ck_state = [s_.cpu().numpy() for s_ in st]
    nh = ga.ga_integrator_history(integ)
    assert nh == (0 if guess == ga.GA_GUESS_ZERO else 4)
    ck_hist = []
    for a in range(nh):
        row = []
        for j in range(k):
            out = torch.empty(nf, dtype=torch.float64, device=DEV)
            ga.ga_stage_solution(integ, j, a, out)
            row.append(out.cpu().numpy())
        ck_hist.append(row)
    integ.close()

    integ = fresh()
    st = [_t(v) for v in ck_state]
    ga.ga_integrator_set_history(integ, [[_t(v) for v in row] for row in ck_hist])
    assert ga.ga_integrator_history(integ) == nh
    ga.ga_step(integ, st, 4)
    for s_, r_ in zip(st, ref):
        assert np.array_equal(s_.cpu().numpy(), r_)
    integ.close()
    if guess == ga.GA_GUESS_ZERO:
        with pytest.raises(ga.GAError):
            ga.ga_integrator_set_history(fresh(), [[_t(ck_state[0]), _t(ck_state[0])]])
