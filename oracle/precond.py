"""The single-patch mass preconditioner of Sec. 5.4 (definition of the
preconditioner with its matrices M-hat, D-hat, D):

    P = D^{1/2} Dhat^{-1/2} Mhat Dhat^{-1/2} D^{1/2},

Mhat = the parametric mass matrix = Kronecker product of the univariate
parametric mass matrices (tensor basis on the unit cube), Dhat = diag(Mhat),
D = diag(M).  With s = (Dhat/D)^{1/2} this gives
P^{-1} r = s * Mhat^{-1} (s * r), and Mhat^{-1} is applied factor by factor
(inverse of a Kronecker product = Kronecker product of the inverses).
All matrices are restricted to the free (Dirichlet-eliminated) coefficients.
"""
import numpy as np
import scipy.linalg as sla

from .operators import parametric_mass_1d


class KronPreconditioner:
    def __init__(self, space, diagM):
        """``diagM``: diag(M) on the free coefficients (co-lex)."""
        self.space = space
        self.Mh = []
        for a in range(space.dim):
            r = slice(space.lo[a], space.m[a] - space.hi[a])
            self.Mh.append(parametric_mass_1d(space.n[a], space.p)[r, r])
        dh = np.diag(self.Mh[0]).copy()
        for a in range(1, space.dim):
            dh = np.kron(np.diag(self.Mh[a]), dh)
        self.Dhat = dh
        self.D = np.asarray(diagM, dtype=np.float64)
        self.s = np.sqrt(self.Dhat / self.D)
        self.chol = [sla.cho_factor(A) for A in self.Mh]

    def kron_solve(self, v):
        """Mhat^{-1} v, solving along one tensor axis at a time."""
        sh = tuple(self.space.mf[::-1])
        t = np.asarray(v, dtype=np.float64).reshape(sh)
        d = self.space.dim
        for a in range(d):
            ax = d - 1 - a  # numpy axis of tensor direction a
            t = np.moveaxis(t, ax, 0)
            t2 = sla.cho_solve(self.chol[a], t.reshape(t.shape[0], -1))
            t = np.moveaxis(t2.reshape(t.shape), 0, ax)
        return t.ravel()

    def apply(self, r):
        """z = P^{-1} r."""
        return self.s * self.kron_solve(self.s * r)

    def dense(self):
        """P itself, formed densely with np.kron (tiny meshes only)."""
        Mh = self.Mh[0]
        for a in range(1, self.space.dim):
            Mh = np.kron(self.Mh[a], Mh)
        sq = np.sqrt(self.D / self.Dhat)
        return sq[:, None] * Mh * sq[None, :]
