"""Pins of the glued multi-patch oracle (oracle/multipatch.py) and of patches
with free (interface) faces."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import multipatch as mp, operators, precond
from paper_2102_11536_amd import workloads


def _deform(g, amp):
    out = g.copy()
    s = np.sin(np.pi * g)
    for c in range(3):
        out[:, c] = g[:, c] + amp * s[:, (c + 1) % 3] * s[:, (c + 2) % 3]
    return out


def test_single_box_is_the_single_patch():
    n, p = 4, 2
    b = mp.Brick((1, 1, 1), n, p)
    ctrl = workloads.brick_ctrl((1, 1, 1), n, p, 0)
    gp = mp.GluedProblem(b, [ctrl])
    sp_ = operators.Space(n, p, 3)
    M, K = operators.free_operators(sp_, ctrl)
    assert abs(gp.M - M).max() <= 1e-15 * abs(M).max()
    assert abs(gp.K - K).max() <= 1e-15 * abs(K).max()
    P = precond.KronPreconditioner(sp_, M.diagonal())
    r = np.random.default_rng(0).standard_normal(b.n_global)
    assert np.allclose(gp.asm_apply(r), P.apply(r), rtol=1e-13, atol=0)


@pytest.mark.parametrize("amp", [0.0, 0.05])
def test_p1_glued_equals_one_patch_of_twice_the_elements(amp):
    # degree-1 B-splines are C^0 anyway: two glued boxes of n elements are one
    # patch of 2n elements with the same nodal control points
    n = 3
    b = mp.Brick((2, 1, 1), n, 1)
    ctrls = [workloads.brick_ctrl((2, 1, 1), n, 1, r, amp=amp) for r in range(2)]
    gp = mp.GluedProblem(b, ctrls)
    sp_ = operators.Space((2 * n, n, n), 1)
    ctrl = _deform(workloads.identity_ctrl((2 * n, n, n), 1, 3), amp)
    M, K = operators.free_operators(sp_, ctrl)
    assert gp.M.shape == M.shape
    assert abs(gp.M - M).max() <= 1e-14 * abs(M).max()
    assert abs(gp.K - K).max() <= 1e-13 * abs(K).max()


@pytest.mark.parametrize("P,nadj", [((2, 1, 1), 2), ((2, 2, 1), 4), ((2, 2, 2), 8), ((3, 1, 1), 2)])
def test_multiplicity(P, nadj):
    b = mp.Brick(P, 3, 2)
    cnt = b.multiplicity()
    assert cnt.max() == nadj and cnt.min() == 1
    # every patch's map is injective and hits the global unknowns
    for r in range(len(b.boxes)):
        g = b.local_to_global(r)
        assert len(np.unique(g)) == len(g) and g.min() >= 0 and g.max() < b.n_global


def test_glued_operators_spd_and_asm_condition():
    # kappa(P_ad^{-1} M) <= C N_adj^2 (Sec. 5.5): bounded growth with the adjacency
    kap = {}
    for P, nadj in (((1, 1, 1), 1), ((2, 1, 1), 2), ((2, 2, 1), 4)):
        b = mp.Brick(P, 3, 2)
        gp = mp.GluedProblem(b, [workloads.brick_ctrl(P, 3, 2, r) for r in range(len(b.boxes))])
        M = gp.M.toarray()
        assert np.allclose(M, M.T, atol=1e-16)
        assert np.linalg.eigvalsh(M).min() > 0
        Pinv = np.column_stack([gp.asm_apply(e) for e in np.eye(b.n_global)])
        assert np.allclose(Pinv, Pinv.T, atol=1e-10 * abs(Pinv).max())
        ev = np.sort(np.real(sla.eigvals(Pinv @ M)))
        kap[P] = ev[-1] / ev[0]
        assert kap[P] <= 2.0 * nadj ** 2, (P, kap[P])
    assert kap[(1, 1, 1)] < kap[(2, 1, 1)] < kap[(2, 2, 1)]


@pytest.mark.parametrize("mask", [0b111101, 0b111110, 0b110011, 0b001111, 0])
def test_free_face_space_and_preconditioner(mask):
    # a patch with free faces: the restriction keeps those coefficients, and the
    # Kronecker preconditioner is the dense solve of its printed product
    n, p = 3, 2
    sp_ = operators.Space(n, p, 3, dirichlet_faces=mask)
    ctrl = workloads.deformed_cube_ctrl(n, p)
    M, _ = operators.free_operators(sp_, ctrl)
    assert M.shape[0] == int(np.prod(sp_.mf))
    P = precond.KronPreconditioner(sp_, M.diagonal())
    r = np.random.default_rng(1).standard_normal(M.shape[0])
    assert np.allclose(P.apply(r), np.linalg.solve(P.dense(), r), rtol=1e-10, atol=1e-12)
    full = operators.Space(n, p, 3, dirichlet_faces=0)
    assert full.n_free == full.n_dof
