"""Conforming (C^0-glued) multi-patch spline spaces and the additive Schwarz
mass preconditioner (Sec. 5.3 multi-patch B-splines, Sec. 5.5 preconditioner
on a multi-patch domain), for a brick of patches.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layout (the workload of the glued cubes): the unit cube split into
P = (P_x, P_y, P_z) boxes, box r = (b_x, b_y, b_z) the patch Omega^(r), every
patch with n elements per direction and degree p (uniform open knot vectors),
each with its own map F^(r).  Along axis a, patch-local coefficient i (0..m-1,
m = n + p) of box b_a has global index g = b_a (m - 1) + i, so the last
coefficient of one box and the first of the next are the same global one (the
conformity assumption of Sec. 5.3: matching knots and control points on the
shared face).  The global grid has P_a (m - 1) + 1 coefficients per axis; the
homogeneous Dirichlet data fix its outer layer, so the unknowns are the global
indices 1 .. P_a (m - 1) - 1, numbered co-lex (x fastest).

Definitions followed:
* G^(r) (local -> global map), J_l, n_l (multiplicity) and N_adj = max n_l;
* the global mass and stiffness matrices M = sum_r G^(r)T M^(r) G^(r) with the
  patch matrices M^(r), K^(r) over the patch's globally free coefficients;
* the additive Schwarz preconditioner
  P_ad^{-1} = sum_r R^(r)T (P^(r))^{-1} R^(r), R^(r) the restriction to the
  global indices J^(r) of patch r and P^(r) the single-patch preconditioner of
  Sec. 5.4 built from M^(r) (its diagonal) and the parametric M-hat^(r) on the
  patch's free index range.
"""
import numpy as np
import scipy.sparse as sp

from . import operators, precond


class Brick:
    def __init__(self, P, n, p):
        self.P = tuple(int(v) for v in P)
        self.n, self.p = int(n), int(p)
        self.m = self.n + self.p
        self.Mg = tuple(b * (self.m - 1) + 1 for b in self.P)   # global coefficients per axis
        self.mfg = tuple(v - 2 for v in self.Mg)                # global unknowns per axis
        self.boxes = [(bx, by, bz) for bz in range(self.P[2]) for by in range(self.P[1])
                      for bx in range(self.P[0])]

    @property
    def n_global(self):
        return int(np.prod(self.mfg))

    def faces(self, r):
        """Dirichlet face mask of patch r: its faces on the outer boundary."""
        b = self.boxes[r]
        mask = 0
        for a in range(3):
            if b[a] == 0:
                mask |= 1 << (2 * a)
            if b[a] == self.P[a] - 1:
                mask |= 1 << (2 * a + 1)
        return mask

    def space(self, r):
        return operators.Space(self.n, self.p, 3, dirichlet_faces=self.faces(r))

    def local_to_global(self, r):
        """G^(r) on the patch's free coefficients (co-lex over its free grid):
        the global unknown index of each."""
        sp_ = self.space(r)
        b = self.boxes[r]
        axes = []
        for a in range(3):
            i = np.arange(sp_.lo[a], self.m - sp_.hi[a])
            axes.append(b[a] * (self.m - 1) + i - 1)              # global unknown index along a
        gx, gy, gz = np.meshgrid(axes[0], axes[1], axes[2], indexing="ij")
        flat = gx + self.mfg[0] * (gy + self.mfg[1] * gz)
        return np.transpose(flat, (2, 1, 0)).ravel()              # co-lex: x fastest

    def multiplicity(self):
        """n_l for every global unknown."""
        cnt = np.zeros(self.n_global, dtype=np.int64)
        for r in range(len(self.boxes)):
            np.add.at(cnt, self.local_to_global(r), 1)
        return cnt


class GluedProblem:
    """Global M and K, the patch operators and the additive Schwarz P_ad."""

    def __init__(self, brick, ctrls):
        self.brick = brick
        N = brick.n_global
        self.maps, self.Ml, self.Kl, self.Pl = [], [], [], []
        M = sp.csr_matrix((N, N))
        K = sp.csr_matrix((N, N))
        for r in range(len(brick.boxes)):
            space = brick.space(r)
            Mr, Kr = operators.free_operators(space, ctrls[r])
            g = brick.local_to_global(r)
            R = sp.csr_matrix((np.ones(len(g)), (np.arange(len(g)), g)), shape=(len(g), N))
            M = M + R.T @ Mr @ R
            K = K + R.T @ Kr @ R
            self.maps.append(g)
            self.Ml.append(Mr)
            self.Kl.append(Kr)
            self.Pl.append(precond.KronPreconditioner(space, Mr.diagonal()))
        self.M, self.K = M.tocsr(), K.tocsr()

    def asm_apply(self, r):
        """P_ad^{-1} r."""
        z = np.zeros(self.brick.n_global)
        for g, P in zip(self.maps, self.Pl):
            np.add.at(z, g, P.apply(r[g]))
        return z
