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


def stratified_rows(mf, p, edges_xy, edges_z, count, seed):
    """Free-coefficient rows of a 3-D patch for sampled checks: each coordinate is
    taken half of the time next to a tile boundary (the coefficients that the
    elements on both sides of an element boundary share, free index b - 1 .. b + p - 2
    for an element boundary b) and otherwise uniformly; the corners of the free box
    are always included.  edges_xy: element boundaries of the xy tiles (both axes),
    edges_z: the boundaries of the z ranges of the workgroups."""
    rng = np.random.default_rng(seed)

    def near(bounds, m):
        out = set()
        for b in bounds:
            for i in range(b - 1, b + p - 1):
                if 0 <= i < m:
                    out.add(i)
        out.update({0, 1, m - 2, m - 1} & set(range(m)))
        return np.array(sorted(out))

    sets = [near(edges_xy, mf[0]), near(edges_xy, mf[1]), near(edges_z, mf[2])]
    rows = set()
    for cx in (0, mf[0] - 1):
        for cy in (0, mf[1] - 1):
            for cz in (0, mf[2] - 1):
                rows.add(cx + mf[0] * (cy + mf[1] * cz))
    while len(rows) < count:
        c = [int(rng.choice(sets[a])) if rng.random() < 0.5 else int(rng.integers(0, mf[a]))
             for a in range(3)]
        rows.add(c[0] + mf[0] * (c[1] + mf[1] * c[2]))
    return np.array(sorted(rows))


def check_step_rows(space, ctrl, rows, L, Ln, tau, k, rho, bar):
    """One step L -> Ln of the order-2k scheme checked on sampled rows with the
    oracle's row-by-row operators: the stage equations M X_j = -K Y_j hold to `bar`
    (relative to max |K Y_j| on the rows), and the update relations of the other
    two vectors of each block hold to 1e-12.  Returns the worst stage residual."""
    T = galpha.predictors(L, tau, k)
    Y = galpha.stage_arguments(L, T, k)
    prm = galpha.block_params(k, rho)
    worst = 0.0
    for j in range(k):
        a = 3 * j
        Xj = T[a] + prm[j][0] * (Ln[a] - T[a])  # X_j = T + alpha P, P = L_new - T
        lhs = operators.sampled_rows(space, ctrl, rows, Xj, "M")
        rhs = -operators.sampled_rows(space, ctrl, rows, Y[j], "K")
        scale = np.max(np.abs(rhs))
        assert scale > 0, j
        err = np.max(np.abs(lhs - rhs)) / scale
        worst = max(worst, err)
        assert err < bar, (j, err)
    for j, (al, be, gm, _) in enumerate(prm):
        a = 3 * j
        Pj = Ln[a] - T[a]
        assert rel(Ln[a - 1], T[a - 1] + gm * tau * Pj) < 1e-12
        assert rel(Ln[a - 2], T[a - 2] + be * tau ** 2 * Pj) < 1e-12
    return worst


# ---- oracle rows in worker processes (large patches) --------------------------

_POOL_STATE = {}


def _pool_init(n, p, ctrl, vectors):
    _POOL_STATE["space"] = operators.Space(n, p, 3)
    _POOL_STATE["ctrl"] = ctrl
    _POOL_STATE["vec"] = vectors


def _pool_task(args):
    name, which, rows = args
    st = _POOL_STATE
    return operators.sampled_rows(st["space"], st["ctrl"], rows, st["vec"][name], which)


def oracle_rows(n, p, ctrl, vectors, requests, workers=8):
    """(A x)_rows of the oracle's row-by-row operators for every request
    (vector name, 'M' | 'K' | 'D', rows), split over `workers` processes started
    fresh (spawn: they import numpy and the oracle only, never the GPU runtime).
    vectors: {name: free-coefficient vector}.  Returns one array per request."""
    import concurrent.futures as cf
    import multiprocessing as mp
    tasks, index = [], []
    for q, (name, which, rows) in enumerate(requests):
        rows = np.asarray(rows)
        for chunk in np.array_split(rows, max(1, min(workers, len(rows) // 8))):
            tasks.append((name, which, chunk))
            index.append(q)
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                initializer=_pool_init, initargs=(n, p, ctrl, vectors)) as ex:
        parts = list(ex.map(_pool_task, tasks))
    out = [[] for _ in requests]
    for q, part in zip(index, parts):
        out[q].append(part)
    return [np.concatenate(o) for o in out]
