"""Shared helpers of the tests: oracle set-ups on the seeded workloads."""
import numpy as np
import scipy.linalg as sla

from oracle import galpha, operators, precond, solvers
from paper_2102_11536_amd import workloads


class OracleProblem:
    def __init__(self, dim, n, p, geometry="deformed", seed=None):
        self.dim, self.n, self.p = dim, n, p
        self.space = operators.Space(n, p, dim)
        self.ctrl = workloads.make_geometry(dim, n, p, geometry, seed)
        self.M, self.K = operators.free_operators(self.space, self.ctrl)
        self.P = precond.KronPreconditioner(self.space, self.M.diagonal())
        self._chol = None

    @property
    def chol(self):
        if self._chol is None:
            self._chol = solvers.CholeskySolver(self.M)
        return self._chol

    def lambda_max(self):
        if self.M.shape[0] <= 3000:
            return float(sla.eigh(self.K.toarray(), self.M.toarray(), eigvals_only=True)[-1])
        from scipy.sparse.linalg import eigsh, LinearOperator
        op = LinearOperator(self.M.shape, matvec=lambda v: self.chol.solve(self.K @ v))
        return float(eigsh(op, k=1, which="LM", return_eigenvectors=False)[0])

    def tau(self, rho=0.5, frac=0.5):
        al, be, ga, _ = galpha.block_params(1, rho)[0]
        theta_s = (16 * al - 8) / (8 * be - 4 * ga)
        return frac * np.sqrt(theta_s / self.lambda_max())

    def run(self, U0, V0, k, rho, tau, nsteps):
        L = galpha.initial_state(U0, V0, k, lambda y: self.K @ y, self.chol.solve)
        out = [L]
        for _ in range(nsteps):
            L = galpha.step(L, tau, k, rho, lambda y: self.K @ y, self.chol.solve)
            out.append(L)
        return out


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
