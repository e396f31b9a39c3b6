"""The 1-D dispersion study (Sec. 6.2): u_tt = omega^2 u_xx on (0, 1) with
homogeneous Dirichlet data and the exact solution u = sin(j pi x) cos(pi t),
omega = 1/j; splines of degree p and regularity C^{p-1} on N uniform
elements (identity map), the order-2k scheme of ``galpha`` with rho_b, rho_s.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions followed:
* the semi-discrete system M U'' + omega^2 K U = 0 (eq. mp with the 1-D
  Galerkin matrices of Sec. 2, K_ij = int b_i' b_j');
* the initial data: U_0 = the L2 projection of sin(j pi x) (M U_0 = f_j with
  f_j,i = int b_i sin(j pi x)), V_0 = 0;
* the error measure: the relative L2(0, 1) error of the displacement at the
  final time, ||u_h - u|| / ||u||, by Gauss quadrature with enough points per
  element for the smooth exact solution;
* reading: a run is only meaningful where every discrete mode is inside the
  stability region, tau^2 omega^2 lambda_max(M^{-1} K) <= Theta_s; at tau = 0.05
  and N = 400, p = 4 that holds for j >= 53 (rho = 0.5), so the study covers
  the stable wavenumbers of each tau (the figure of Sec. 6.2 is not available).
"""
import numpy as np
from . import bspline, galpha, operators, solvers


class Wave1D:
    def __init__(self, N, p):
        self.N, self.p = int(N), int(p)
        self.space = operators.Space(self.N, self.p, dim=1)
        t = bspline.open_uniform_knots(self.N, self.p)
        m = self.N + self.p
        grev = np.array([np.mean(t[i + 1:i + self.p + 1]) for i in range(m)])
        ctrl = grev[:, None]                  # identity map: Greville abscissae (linear precision)
        self.M, self.K = operators.free_operators(self.space, ctrl)
        self.chol = solvers.CholeskySolver(self.M)
        # fine quadrature for the load vectors and the error: 2p + 8 points per element
        self.xq, self.wq, Bq, _ = bspline.tables_1d(self.N, self.p, nq=2 * self.p + 8)
        self.Bq = Bq[:, self.space.free_index()]          # [points][free]

    @property
    def n_free(self):
        return self.M.shape[0]

    def load(self, j):
        """f_i = int_0^1 b_i sin(j pi x) dx."""
        return self.Bq.T @ (self.wq * np.sin(j * np.pi * self.xq))

    def projection(self, j):
        return self.chol.solve(self.load(j))

    def rel_l2_error(self, U, j, t):
        """||u_h(., t) - sin(j pi x) cos(pi t)|| / ||sin(j pi x) cos(pi t)||."""
        ex = np.sin(j * np.pi * self.xq) * np.cos(np.pi * t)
        uh = self.Bq @ U
        return float(np.sqrt(np.sum(self.wq * (uh - ex) ** 2) / np.sum(self.wq * ex ** 2)))

    def run(self, j, k, rho, tau, nsteps, rho_s=None):
        """Displacement after nsteps steps from the projected data (omega = 1/j)."""
        w2 = 1.0 / j ** 2
        K = self.K
        apply_K = lambda y: w2 * (K @ y)
        U0 = self.projection(j)
        L = galpha.initial_state(U0, 0 * U0, k, apply_K, self.chol.solve)
        for _ in range(nsteps):
            L = galpha.step(L, tau, k, rho, apply_K, self.chol.solve, rho_s=rho_s)
        return L[-2]

    def discrete_eigenvalues(self):
        """Generalized eigenvalues of (K, M), ascending."""
        import scipy.linalg as sla
        return sla.eigh(self.K.toarray(), self.M.toarray(), eigvals_only=True)


def stability_limit_closed(rho, rho_s=None):
    """Theta_s of the family (rho_b = rho, rho_s): the lambda = -1 root of the
    type-k characteristic polynomial, (4 alpha - 2) / (2 beta - gamma) (the
    reading of the printed Omega_s used throughout; the same for every k)."""
    a, b, g, _ = galpha.block_params(1, rho, rho_s)[0]
    return (4 * a - 2) / (2 * b - g)


def smallest_stable_j(lam_max, rho, tau, rho_s=None):
    """Smallest wavenumber j whose run is stable: tau^2 lambda_max / j^2 <= Theta_s
    (every discrete mode of M^{-1} omega^2 K inside the stability region)."""
    return max(1, int(np.ceil(np.sqrt(tau ** 2 * lam_max / stability_limit_closed(rho, rho_s)) - 1e-12)))
