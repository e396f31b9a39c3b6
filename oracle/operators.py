"""Mass and stiffness matrices of a single tensor-product spline patch, by
Gauss quadrature, with homogeneous Dirichlet elimination.

Definitions followed:
* Tensor-product basis and co-lexicographic numbering, x fastest (Sec. 5.1-5.2):
  with C-ordered arrays of shape [m_z, m_y, m_x] the flat index is co-lex, and
  the d-variate basis matrix is kron(B_z, B_y, B_x).
* Isoparametric geometry F(xi) = sum_i C_i B_i(xi) (Sec. 5.2), J = DF.
* Mass matrix (eq. mass_matrix): M_ij = int B_i B_j |det DF| d xi.
* Stiffness matrix (eq. pde with omega = 1, giving K in eq. mp; not written out
  in the paper): K_ij = int grad B_i . grad B_j dx
                      = int gradhat B_i^T (|det J| J^{-1} J^{-T}) gradhat B_j d xi.
* Homogeneous Dirichlet data (second remark of Sec. 2): the unknowns are the
  coefficients of basis functions that vanish on the boundary, i.e. all
  indices 1 <= i_a <= m_a - 2 (0-based) in every direction.  A patch of a
  glued multi-patch domain (Sec. 5.3) keeps the coefficients of its interface
  faces: there the range starts at 0 or ends at m_a - 1.
* Assumption 3 (det DF >= delta > 0) is checked at every quadrature point.

The sums over quadrature points are written as sparse products
B^T diag(W) B of the tensor basis matrices; no blocking or sum factorisation.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline


class Space:
    """Spline space of degree p on n_a uniform elements per direction of the
    unit square/cube, with the 1-D tables of ``bspline.tables_1d``.

    ``dirichlet_faces``: bit 2a marks the face xi_a = 0, bit 2a+1 the face
    xi_a = 1 as carrying the homogeneous Dirichlet data (default: all faces);
    along axis a the free coefficients are lo[a] .. m[a]-1-hi[a]."""

    def __init__(self, n, p, dim=None, dirichlet_faces=None):
        if np.isscalar(n):
            n = (int(n),) * (dim if dim is not None else 3)
        self.n = tuple(int(v) for v in n)  # (n_x, n_y[, n_z])
        self.dim = len(self.n)
        self.p = int(p)
        self.m = tuple(v + self.p for v in self.n)
        mask = (1 << (2 * self.dim)) - 1 if dirichlet_faces is None else int(dirichlet_faces)
        self.lo = tuple((mask >> (2 * a)) & 1 for a in range(self.dim))
        self.hi = tuple((mask >> (2 * a + 1)) & 1 for a in range(self.dim))
        self.mf = tuple(self.m[a] - self.lo[a] - self.hi[a] for a in range(self.dim))
        self.tabs = [bspline.tables_1d(v, self.p) for v in self.n]  # per axis x, y, z

    @property
    def n_dof(self):
        return int(np.prod(self.m))

    @property
    def n_free(self):
        return int(np.prod(self.mf))

    def free_index(self):
        """Flat co-lex indices (full numbering) of the free coefficients, in
        co-lex order of the free grid."""
        idx = np.arange(self.n_dof).reshape(self.m[::-1])
        sl = tuple(slice(self.lo[a], self.m[a] - self.hi[a]) for a in reversed(range(self.dim)))
        return idx[sl].ravel()

    def to_full(self, x_free):
        x = np.zeros(self.n_dof)
        x[self.free_index()] = x_free
        return x


def _kron_all(mats_xyz):
    """kron(A_z, A_y, A_x) for matrices given in axis order x, y[, z]."""
    out = sp.csr_matrix(mats_xyz[0])
    for a in mats_xyz[1:]:
        out = sp.kron(sp.csr_matrix(a), out, format="csr")
    return out


def _ops(space, qsel=None, dsel=None):
    """Tensor basis matrix and its d partial derivatives, optionally restricted
    to 1-D quadrature-point ranges ``qsel[a]`` and basis ranges ``dsel[a]``."""
    Bs, Ds, ws = [], [], []
    for a in range(space.dim):
        _, wq, B, D = space.tabs[a]
        qs = slice(None) if qsel is None else qsel[a]
        ds = slice(None) if dsel is None else dsel[a]
        Bs.append(B[qs, ds])
        Ds.append(D[qs, ds])
        ws.append(wq[qs])
    Bt = _kron_all(Bs)
    grads = []
    for a in range(space.dim):
        mats = [Ds[b] if b == a else Bs[b] for b in range(space.dim)]
        grads.append(_kron_all(mats))
    w = ws[0]
    for v in ws[1:]:
        w = np.kron(v, w)
    return Bt, grads, w


def geometry_factors(space, ctrl, qsel=None, dsel=None):
    """At every quadrature point: W = w |det J| and G = w |det J| J^{-1} J^{-T}.

    ``ctrl`` holds the control points [N_dof, dim] in co-lex order (or, with
    ``dsel``, those of the selected basis box).  Raises ValueError when
    det J <= 0 anywhere (Assumption 3)."""
    Bt, grads, w = _ops(space, qsel, dsel)
    d = space.dim
    J = np.empty((Bt.shape[0], d, d))
    for a in range(d):
        J[:, :, a] = grads[a] @ ctrl  # dF_c / dxi_a
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("geometry map is not orientation-preserving (det DF <= 0)")
    Jinv = np.linalg.inv(J)
    W = w * det
    G = W[:, None, None] * np.einsum("qij,qkj->qik", Jinv, Jinv)
    return Bt, grads, W, G


def assemble(space, ctrl):
    """Full (boundary included) sparse M and K [N_dof, N_dof] by quadrature."""
    Bt, grads, W, G = geometry_factors(space, ctrl)
    M = (Bt.T @ sp.diags(W) @ Bt).tocsr()
    K = None
    for a in range(space.dim):
        for b in range(space.dim):
            t = grads[a].T @ sp.diags(G[:, a, b]) @ grads[b]
            K = t if K is None else K + t
    return M, K.tocsr()


def restrict(space, A):
    """Dirichlet elimination: the free-by-free block of a full matrix."""
    f = space.free_index()
    return A[f][:, f].tocsr()


def free_operators(space, ctrl):
    """(M, K) on the free coefficients, as CSR matrices."""
    M, K = assemble(space, ctrl)
    return restrict(space, M), restrict(space, K)


def parametric_mass_1d(n, p):
    """Univariate parametric mass matrix [m, m] (M-hat factor, Sec. 5.4):
    int_0^1 b_i b_j by the same Gauss rule (exact for degree 2p)."""
    _, wq, B, _ = bspline.tables_1d(n, p)
    return B.T @ (wq[:, None] * B)


def parametric_stiffness_1d(n, p):
    """Univariate int_0^1 b_i' b_j' (used only by tests)."""
    _, wq, _, D = bspline.tables_1d(n, p)
    return D.T @ (wq[:, None] * D)


def sampled_rows(space, ctrl, rows_free, x_free, which):
    """(A x)_i for a few free rows i without assembling A (A = 'M' or 'K'):
    the quadrature sum restricted to the support of B_i, which is exactly the
    definition since B_i vanishes elsewhere.  Used at sizes where assembly
    does not fit."""
    p, d = space.p, space.dim
    x_full = space.to_full(x_free)
    f = space.free_index()
    out = np.empty(len(rows_free))
    shape_rev = space.m[::-1]
    for s, r in enumerate(rows_free):
        gi = f[r]
        mi = np.unravel_index(gi, shape_rev)[::-1]  # (ix, iy, iz)
        qsel, dsel, loc = [], [], []
        for a in range(d):
            e0 = max(mi[a] - p, 0)
            e1 = min(mi[a], space.n[a] - 1)
            nq = p + 1
            qsel.append(slice(e0 * nq, (e1 + 1) * nq))
            b0 = e0
            b1 = min(e1 + p, space.m[a] - 1)
            dsel.append(slice(b0, b1 + 1))
            loc.append(mi[a] - b0)
        box = np.ix_(*[np.arange(s_.start, s_.stop) for s_ in dsel[::-1]])
        c_full = ctrl.reshape(*shape_rev, d)
        cbox = c_full[box].reshape(-1, d)
        xbox = x_full.reshape(shape_rev)[box].ravel()
        Bt, grads, W, G = geometry_factors(space, cbox, qsel, dsel)
        dims = [s_.stop - s_.start for s_ in dsel]
        li = 0
        stride = 1
        for a in range(d):
            li += loc[a] * stride
            stride *= dims[a]
        col = lambda A: A[:, [li]].toarray().ravel()
        if which == "M":
            out[s] = col(Bt) @ (W * (Bt @ xbox))
        elif which == "K":
            gx = [g @ xbox for g in grads]
            out[s] = sum(col(grads[a]) @ (G[:, a, b] * gx[b])
                         for a in range(d) for b in range(d))
        else:  # 'D': the diagonal entry M_ii
            out[s] = (col(Bt) ** 2) @ W
    return out
