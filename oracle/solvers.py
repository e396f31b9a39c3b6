"""Mass solves: preconditioned conjugate gradients (the solver of Sec. 5 and 6)
and direct Cholesky factorisations of the assembled M.

Reading of the PCG stopping rule (the paper gives only the tolerance 1e-12 and
the zero initial guess, Sec. 6): iterate until sqrt(r^T z) <= tol *
sqrt(b^T P^{-1} b), where z = P^{-1} r, i.e. the preconditioned residual norm
relative to that of the right-hand side (not of the initial residual), so a
better initial guess can only shorten the iteration.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def pcg(apply_A, b, apply_Pinv, x0=None, tol=1e-12, maxit=1000):
    """Textbook PCG.  Returns (x, iterations, converged)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.sqrt(max(float(b @ apply_Pinv(b)), 0.0))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, True
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = apply_Pinv(r)
    rz = float(r @ z)
    p = z.copy()
    it = 0
    while True:
        if np.sqrt(max(rz, 0.0)) <= tol * bnorm:
            return x, it, True
        if it >= maxit:
            return x, it, False
        q = apply_A(p)
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = apply_Pinv(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        p = z + beta * p
        rz = rz_new
        it += 1


class CholeskySolver:
    """Direct solve with a Cholesky factor of the assembled (free) M: dense
    LAPACK for small systems, banded LAPACK (co-lex bandwidth) otherwise."""

    def __init__(self, M, dense_limit=6000):
        M = sp.csr_matrix(M)
        n = M.shape[0]
        if n <= dense_limit:
            self.kind = "dense"
            self.f = sla.cho_factor(M.toarray(), lower=True)
        else:
            self.kind = "banded"
            coo = M.tocoo()
            u = int(np.max(coo.col - coo.row))
            ab = np.zeros((u + 1, n))
            sel = coo.col >= coo.row
            r, c, v = coo.row[sel], coo.col[sel], coo.data[sel]
            ab[u + r - c, c] = v
            self.u = u
            self.f = sla.cholesky_banded(ab, lower=False)

    def solve(self, b):
        if self.kind == "dense":
            return sla.cho_solve(self.f, b)
        return sla.cho_solve_banded((self.f, False), b)
