"""Batched independent patches (one launch per degree / pass / vector op, PCG
iterations replayed from a captured hipGraph) against the oracle and against
the same patches stepped one at a time."""
import sys

import numpy as np
import pytest
import torch

from paper_2102_11536_amd import ga, workloads
from tests.helpers import OracleProblem, check_step_rows, rel, stratified_rows

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


def _setup(specs):
    pts, U0s = [], []
    for (n, p, gseed, useed) in specs:
        pts.append(ga.ga_setup_patch(3, n, p, workloads.smooth_random_ctrl(n, p, gseed)))
        U0s.append(workloads.grf(n, p, seed=useed))
    return pts, U0s


def _tau(pts, rho=0.5):
    lam = max(ga.ga_lambda_max(pt, 30) for pt in pts)
    return 0.5 * np.sqrt(ga.ga_stability_limit(rho) / lam)


def _run_batch(pts, U0s, k, tau, nsteps, use_graph=True, tune=False, rtol=1e-12, prec=ga.GA_FP64):
    b = ga.ga_batch_create(pts, k, 0.5, tau, rtol=rtol)
    if prec != ga.GA_FP64:
        ga.ga_batch_set_precision(b, prec)
    if tune:
        ga.ga_batch_tune(b, reps=2)
    U = _t(np.concatenate(U0s))
    state = [torch.zeros(b.n_total, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_batch_init_state(b, U, torch.zeros_like(U), state)
    hist = [[_np(s) for s in state]]
    its = []
    for _ in range(nsteps):
        its.append(ga.ga_batch_step(b, state, 1, use_graph=use_graph))
        hist.append([_np(s) for s in state])
    return b, hist, np.concatenate(its)


def _split(b, v):
    return [v[o:o + pt.n_free] for o, pt in zip(b.offsets, b.patches)]


SMALL = [(4, 2, 11, 111), (5, 3, 12, 112), (3, 4, 13, 113), (6, 2, 14, 114)]


def test_batch_matches_oracle():
    _say("batch vs oracle")
    k = 2
    pts, U0s = _setup(SMALL)
    tau = _tau(pts)
    b, hist, its = _run_batch(pts, U0s, k, tau, 8)
    assert ga.ga_batch_graph_replays(b) > 0
    for r, (n, p, gseed, _) in enumerate(SMALL):
        pr = OracleProblem(3, n, p, geometry="random", seed=gseed)
        ora = pr.run(U0s[r], 0 * U0s[r], k, 0.5, tau, 8)
        M = pr.M
        for step in (1, 4, 8):
            for s in range(3 * k):
                g = _split(b, hist[step][s])[r]
                o = ora[step][s - 2]
                d = g - o
                # fields that are exactly zero (e.g. L^3 after one step from V0 = 0) compare absolutely
                e = np.sqrt(d @ (M @ d)) / max(np.sqrt(o @ (M @ o)), 1e-300)
                assert e < 1e-10, (r, step, s, e)
    _say("  iterations per system", its.mean(axis=0).tolist())


def test_batch_equals_separate_patches():
    # uneven batch of the multi-patch recipe at reduced sizes; every patch must
    # follow the single-patch integrator
    specs = workloads.multipatch_specs(R=12, n_min=4, n_max=14, seed=3)
    _say("batch vs separate", specs)
    k = 2
    pts, U0s = _setup(specs)
    tau = _tau(pts)
    b, hist, _ = _run_batch(pts, U0s, k, tau, 6, tune=True)
    for r, pt in enumerate(pts):
        integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12)
        state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        U = _t(U0s[r])
        ga.ga_init_state(integ, U, torch.zeros_like(U), state)
        ga.ga_step(integ, state, 6)
        for s in range(3 * k):
            assert rel(_split(b, hist[-1][s])[r], _np(state[s])) < 1e-10, (r, s)


def test_graph_replays_match_eager():
    # every replay of the captured PCG iteration against the eager launches,
    # with eager work and synchronisations between replays (each step replays
    # the graph several times, and steps are compared one by one)
    _say("graph vs eager")
    k = 2
    pts, U0s = _setup(SMALL[:3])
    tau = _tau(pts)
    bg, hg, ig = _run_batch(pts, U0s, k, tau, 6, use_graph=True)
    be, he, ie = _run_batch(pts, U0s, k, tau, 6, use_graph=False)
    assert ga.ga_batch_graph_replays(bg) >= 6 and ga.ga_batch_graph_replays(be) == 0
    # the order of the FP64 atomic additions may differ between the two runs, so a
    # residual right at the tolerance may take one iteration more in one of them
    assert np.max(np.abs(ig - ie)) <= 1
    for step in range(1, 7):
        for s in range(3 * k):
            # same launches; only the run-to-run order of the FP64 atomic additions differs
            assert rel(hg[step][s], he[step][s]) < 1e-11, (step, s)


def test_batch_per_patch_time_steps():
    # every patch at half its own stability limit: the batch equals the single-patch
    # integrators run with those time steps
    specs = workloads.multipatch_specs(R=6, n_min=4, n_max=12, seed=9)
    k = 2
    pts, U0s = _setup(specs)
    taus = [0.5 * np.sqrt(ga.ga_stability_limit(0.5) / ga.ga_lambda_max(pt, 30)) for pt in pts]
    assert max(taus) > 1.2 * min(taus)
    b = ga.ga_batch_create(pts, k, 0.5, min(taus), rtol=1e-12)
    ga.ga_batch_set_tau(b, taus)
    U = _t(np.concatenate(U0s))
    state = [torch.zeros(b.n_total, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_batch_init_state(b, U, torch.zeros_like(U), state)
    ga.ga_batch_step(b, state, 5)
    got = [_np(s) for s in state]
    for r, pt in enumerate(pts):
        integ = ga.ga_integrator_create(pt, k, 0.5, taus[r], rtol=1e-12)
        st = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        u = _t(U0s[r])
        ga.ga_init_state(integ, u, torch.zeros_like(u), st)
        ga.ga_step(integ, st, 5)
        for s in range(3 * k):
            assert rel(_split(b, got[s])[r], _np(st[s])) < 1e-10, (r, s)
    with pytest.raises(ga.GAError):
        ga.ga_batch_set_tau(b, [1.0] * (len(pts) - 1) + [-1.0])


# ---- FP32 inner PCG inside FP64 refinement, batched (an addition to the paper) ----

def test_batch_mixed_matches_oracle():
    _say("mixed batch vs oracle")
    k = 2
    pts, U0s = _setup(SMALL)
    tau = _tau(pts)
    b, hist, its = _run_batch(pts, U0s, k, tau, 8, prec=ga.GA_FP32)
    assert ga.ga_batch_graph_replays(b) > 0
    worst = 0.0
    for r, (n, p, gseed, _) in enumerate(SMALL):
        pr = OracleProblem(3, n, p, geometry="random", seed=gseed)
        ora = pr.run(U0s[r], 0 * U0s[r], k, 0.5, tau, 8)
        M = pr.M
        for step in (1, 4, 8):
            for s in range(3 * k):
                g = _split(b, hist[step][s])[r]
                o = ora[step][s - 2]
                d = g - o
                e = np.sqrt(d @ (M @ d)) / max(np.sqrt(o @ (M @ o)), 1e-300)
                worst = max(worst, e)
                # the refinement reaches the FP64 tolerance; FP32 enters only the corrections
                assert e < 1e-10, (r, step, s, e)
    _say("  worst M-norm error", worst, "inner iterations per system", its.mean(axis=0).tolist())


def test_batch_mixed_equals_separate_mixed_patches():
    specs = workloads.multipatch_specs(R=8, n_min=4, n_max=12, seed=5)
    _say("mixed batch vs separate", specs)
    k = 2
    pts, U0s = _setup(specs)
    tau = _tau(pts)
    b, hist, _ = _run_batch(pts, U0s, k, tau, 5, tune=True, prec=ga.GA_FP32)
    for r, pt in enumerate(pts):
        integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12, prec=ga.GA_FP32)
        state = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
        U = _t(U0s[r])
        ga.ga_init_state(integ, U, torch.zeros_like(U), state)
        ga.ga_step(integ, state, 5)
        for s in range(3 * k):
            # both stop at relative tolerance 1e-12 by different FP32 paths
            assert rel(_split(b, hist[-1][s])[r], _np(state[s])) < 1e-10, (r, s)


def test_batch_mixed_graph_matches_eager():
    _say("mixed graph vs eager")
    k = 2
    pts, U0s = _setup(SMALL[:3])
    tau = _tau(pts)
    bg, hg, ig = _run_batch(pts, U0s, k, tau, 5, use_graph=True, prec=ga.GA_FP32)
    be, he, ie = _run_batch(pts, U0s, k, tau, 5, use_graph=False, prec=ga.GA_FP32)
    assert ga.ga_batch_graph_replays(bg) >= 5 and ga.ga_batch_graph_replays(be) == 0
    assert np.max(np.abs(ig - ie)) <= 1   # atomic order (see the FP64 test)
    for step in range(1, 6):
        for s in range(3 * k):
            # same launches; only the run-to-run order of the FP64 atomic additions differs
            assert rel(hg[step][s], he[step][s]) < 1e-11, (step, s)


def test_batch_precision_switch_back():
    # FP32 then FP64 again on the same batch: the FP64 solve is the plain one
    k = 2
    pts, U0s = _setup(SMALL[:2])
    tau = _tau(pts)
    b0, h0, _ = _run_batch(pts, U0s, k, tau, 3)
    b = ga.ga_batch_create(pts, k, 0.5, tau, rtol=1e-12)
    ga.ga_batch_set_precision(b, ga.GA_FP32)
    ga.ga_batch_set_precision(b, ga.GA_FP64)
    U = _t(np.concatenate(U0s))
    state = [torch.zeros(b.n_total, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_batch_init_state(b, U, torch.zeros_like(U), state)
    ga.ga_batch_step(b, state, 3)
    for s in range(3 * k):
        # same FP64 launches; shared coefficients are summed by atomics, so the
        # order of the additions (and the last bits) may differ between runs
        assert rel(_np(state[s]), h0[-1][s]) < 1e-12
    with pytest.raises(ga.GAError):
        ga.ga_batch_set_precision(b, 7)


def test_batch_errors():
    pt2 = ga.ga_setup_patch(2, 6, 2, workloads.identity_ctrl(6, 2, 2))
    pt3 = ga.ga_setup_patch(3, 4, 1, workloads.deformed_cube_ctrl(4, 1))
    for bad in ([pt2], [pt3]):
        with pytest.raises(ga.GAError):
            ga.ga_batch_create(bad, 2, 0.5, 1e-3)
    ok = ga.ga_setup_patch(3, 4, 2, workloads.deformed_cube_ctrl(4, 2))
    with pytest.raises(ga.GAError):
        ga.ga_batch_create([ok], 5, 0.5, 1e-3)


def test_batch_long_axes_match_oracle():
    # patches whose free axes fall in the larger register classes of the batched
    # preconditioner passes (65..144 and 145..256 coefficients, along x, y and z),
    # with a small cube: FP64 and mixed batches against the oracle's trajectories
    specs = [((70, 3, 3), 2, 21, 121), ((3, 99, 3), 3, 22, 122), ((3, 3, 150), 2, 23, 123),
             ((160, 3, 2), 4, 24, 124), (4, 3, 25, 125)]
    _say("batch long axes", specs)
    k = 2
    pts, U0s = _setup(specs)
    tau = _tau(pts)
    ora = [OracleProblem(3, n, p, geometry="random", seed=gseed) for (n, p, gseed, _) in specs]
    traj = [pr.run(U0s[r], 0 * U0s[r], k, 0.5, tau, 4) for r, pr in enumerate(ora)]
    for prec in (ga.GA_FP64, ga.GA_FP32):
        b, hist, its = _run_batch(pts, U0s, k, tau, 4, tune=True, prec=prec)
        worst = 0.0
        for r, pr in enumerate(ora):
            M = pr.M
            for step in (1, 4):
                for s in range(3 * k):
                    g = _split(b, hist[step][s])[r]
                    o = traj[r][step][s - 2]
                    d = g - o
                    e = np.sqrt(d @ (M @ d)) / max(np.sqrt(o @ (M @ o)), 1e-300)
                    worst = max(worst, e)
                    # the (160, 3, 2) p = 4 patch sets tau (the smallest step of the
                    # batch) and has the worst-conditioned M; its derivative fields
                    # reach 1.3e-10 after 4 steps of PCG at rtol 1e-12
                    assert e < 1e-9, (prec, r, step, s, e)
            # the same patch alone through the single-patch integrator (banded
            # preconditioner, no tile queue)
            pt = pts[r]
            integ = ga.ga_integrator_create(pt, k, 0.5, tau, rtol=1e-12, prec=prec)
            st = [torch.zeros(pt.n_free, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
            u = _t(U0s[r])
            ga.ga_init_state(integ, u, torch.zeros_like(u), st)
            ga.ga_step(integ, st, 4)
            for s in range(3 * k):
                assert rel(_split(b, hist[4][s])[r], _np(st[s])) < 1e-10, (prec, r, s)
        _say("  prec", prec, "worst M-norm error vs oracle", worst,
             "iterations per system", its.mean(axis=0).tolist())


@pytest.mark.parametrize("prec", [ga.GA_FP64, ga.GA_FP32])
def test_batch_full_size_multipatch(prec):
    # the batched workload at its real sizes (12 patches, 16..96 elements per axis,
    # p in 2..4; free axes 20..93, so both register classes of the batched
    # preconditioner run), in the configuration the bench times: autotuned tile
    # queues, captured iterations, rtol 1e-10.  Two steps; every patch is compared
    # with its single-patch integrator and, on stratified rows, with the oracle's
    # stage equations.
    specs = workloads.multipatch_specs(R=12, n_min=16, n_max=96, seed=7)
    _say("batch full size", prec, specs)
    k, rho, rtol = 2, 0.5, 1e-10
    pts, U0s = _setup(specs)
    tau = _tau(pts)
    b = ga.ga_batch_create(pts, k, rho, tau, rtol=rtol)
    if prec != ga.GA_FP64:
        ga.ga_batch_set_precision(b, prec)
    ga.ga_batch_tune(b, reps=2)
    U = _t(np.concatenate(U0s))
    state = [torch.zeros(b.n_total, dtype=torch.float64, device=DEV) for _ in range(3 * k)]
    ga.ga_batch_init_state(b, U, torch.zeros_like(U), state)
    ga.ga_batch_step(b, state, 1, use_graph=True)
    L = [_np(s_) for s_ in state]
    its = ga.ga_batch_step(b, state, 1, use_graph=True)
    Ln = [_np(s_) for s_ in state]
    _say("  iterations per system", np.asarray(its).ravel().tolist())
    from oracle import operators
    for r, pt in enumerate(pts):
        n, p, gseed, _ = specs[r]
        # the single-patch integrator from the same state, same tau and tolerance
        integ = ga.ga_integrator_create(pt, k, rho, tau, rtol=rtol, prec=prec)
        st = [_t(_split(b, L[s_])[r]) for s_ in range(3 * k)]
        ga.ga_step(integ, st, 1)
        for s_ in range(3 * k):
            e = rel(_split(b, Ln[s_])[r], _np(st[s_]))
            assert e < 1e-8, (r, s_, e)   # two PCG solves, each within rtol 1e-10 of the exact one
        if prec != ga.GA_FP64:
            continue
        # the oracle's stage equations on stratified rows
        ctrl = workloads.smooth_random_ctrl(n, p, gseed)
        sp_ = operators.Space(n, p, 3)
        te = 4 if p <= 3 else 3
        rows = stratified_rows(pt.mf, p, list(range(te, n, te)), list(range(4, n, 4)), 16, r)
        La = {a: _split(b, L[a + 2])[r] for a in range(-2, 3 * k - 2)}
        Lb = {a: _split(b, Ln[a + 2])[r] for a in range(-2, 3 * k - 2)}
        w = check_step_rows(sp_, ctrl, rows, La, Lb, tau, k, rho, 1e-8)
        _say("  patch", r, (n, p), "stage residual on rows", w)
