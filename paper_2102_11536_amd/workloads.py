"""Seeded synthetic workloads: geometry control points and initial data.

This module is shared by the HIP path and the CPU oracle and holds none of the
method's arithmetic (no basis evaluation, quadrature, operators, solves or time
stepping); it only builds input arrays.  Recipes:

* Control points are a map evaluated at the Greville abscissae (knot averages)
  of the open uniform knot vector.  For the identity map this reproduces the
  identity exactly (linear precision of B-splines); for the deformed cube
  x_c = xi_c + a sin(pi xi_{c+1}) sin(pi xi_{c+2}) (cyclic c) it gives a spline
  approximation of that map with det J > 0.
* Gaussian random field (GRF) initial displacement on the free coefficient
  grid: separable squared-exponential covariance with correlation length ell
  at the free Greville abscissae, sampled as (L_z x L_y x L_x) g with
  L = V sqrt(Lambda) from eigh of the 1-D covariance and g ~ N(0, 1) from
  numpy's PCG64 seeded generator, tapered by prod sin(pi x_a) and scaled to
  RMS 1.
* The 2-D standing wave u0 = sin(pi x) sin(pi y) is sampled at the Greville
  abscissae of the free coefficients.
* Glued brick of patches: the unit cube split into P_x x P_y x P_z boxes, each a
  patch with n elements and degree p; the control points of box r are its
  Greville points mapped affinely into the box and then deformed by the global
  map x_c + a sin(pi x_{c+1}) sin(pi x_{c+2}) (so the shared faces match); the
  initial field is a GRF at the global coefficients' Greville-like points.
* Batched multi-patch workload: R independent cube patches, each with a
  seeded element count n_r drawn uniformly from [n_min, n_max], degree p_r
  from {2, 3, 4} and its own smooth random geometry map (seed base + r),
  and a GRF initial displacement per patch (seed base + 100 + r).
* Random parameters of the learned-guess net: normal weights with He scaling
  sqrt(2 / fan_in) and normal biases of standard deviation 0.05, seeded.
"""
import numpy as np


def greville(n, p):
    """Greville abscissae of the open uniform knot vector with n elements and
    degree p (length n + p)."""
    kn = np.concatenate([np.zeros(p + 1), np.arange(1, n) / n, np.ones(p + 1)])
    m = n + p
    if p == 0:
        return 0.5 * (kn[:m] + kn[1:m + 1])
    return np.array([kn[i + 1:i + p + 1].mean() for i in range(m)])


def _grid(axes):
    """Tensor grid of 1-D coordinate arrays (axis order x, y[, z]) as [N, d]
    in co-lex order (x fastest)."""
    mesh = np.meshgrid(*axes[::-1], indexing="ij")  # z, y, x
    return np.stack([mesh[::-1][a].ravel() for a in range(len(axes))], axis=1)


def _ns(n, dim):
    return (int(n),) * dim if np.isscalar(n) else tuple(int(v) for v in n)


def identity_ctrl(n, p, dim):
    ns = _ns(n, dim)
    return _grid([greville(v, p) for v in ns])


def deformed_cube_ctrl(n, p, amp=0.1, dim=3):
    ns = _ns(n, dim)
    g = identity_ctrl(ns, p, dim)
    out = g.copy()
    s = np.sin(np.pi * g)
    for c in range(dim):
        prod = np.ones(len(g))
        for o in range(1, dim):
            prod = prod * s[:, (c + o) % dim]
        out[:, c] = g[:, c] + amp * prod
    return out


def smooth_random_ctrl(n, p, seed, amp=0.06, dim=3):
    """Seeded smooth map: identity plus, per coordinate, two products of sines
    with random integer frequencies (1 or 2) and random amplitudes."""
    ns = _ns(n, dim)
    rng = np.random.default_rng(seed)
    g = identity_ctrl(ns, p, dim)
    out = g.copy()
    for c in range(dim):
        for _ in range(2):
            fr = rng.integers(1, 3, size=dim)
            a = amp * rng.uniform(-1.0, 1.0)
            prod = np.ones(len(g))
            for o in range(dim):
                if o != c:
                    prod = prod * np.sin(np.pi * fr[o] * g[:, o])
            out[:, c] += a * prod
    return out


def grf(n, p, seed, ell=0.1, dim=3):
    """Seeded GRF on the free coefficient grid, shape [N_free] co-lex."""
    ns = _ns(n, dim)
    return grf_on_axes([greville(v, p)[1:-1] for v in ns], seed, ell)


def grf_on_axes(axes, seed, ell=0.1):
    """Seeded GRF on the tensor grid of the given per-axis coordinates (x first),
    co-lex, tapered by prod sin(pi x_a) and scaled to RMS 1."""
    dim = len(axes)
    rng = np.random.default_rng(seed)
    Ls = []
    for x in axes:
        C = np.exp(-0.5 * ((x[:, None] - x[None, :]) / ell) ** 2)
        lam, V = np.linalg.eigh(C)
        Ls.append(V * np.sqrt(np.clip(lam, 0.0, None))[None, :])
    g = rng.standard_normal(tuple(len(x) for x in axes[::-1]))  # [z, y, x]
    for a in range(dim):
        ax = dim - 1 - a
        g = np.moveaxis(np.tensordot(Ls[a], g, axes=([1], [ax])), 0, ax)
    taper = np.ones(1)
    for x in axes:
        taper = np.kron(np.sin(np.pi * x), taper)
    u = g.ravel() * taper
    return u / np.sqrt(np.mean(u * u))


def standing_wave_u0(n, p):
    """sin(pi x) sin(pi y) at the free Greville abscissae (2-D)."""
    ns = _ns(n, 2)
    axes = [greville(v, p)[1:-1] for v in ns]
    pts = _grid(axes)
    return np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1])


# Workload presets (sizes and seeds).  tau is set from the stability limit by
# the caller (0.5 of the critical step).
PRESETS = {
    "wave2d_p2_n32_k1": dict(dim=2, n=32, p=2, k=1, rho=0.5, steps=200,
                             geometry="identity", init="standing_wave"),
    "cube_p3_n64_k2": dict(dim=3, n=64, p=3, k=2, rho=0.5, steps=100, rtol=1e-10,
                           geometry="deformed", init="grf", seed=0),
    "cube_p4_n128_k3": dict(dim=3, n=128, p=4, k=3, rho=0.5, steps=100,
                            geometry="deformed", init="grf", seed=1),
    "cube_p3_n128_k2": dict(dim=3, n=128, p=3, k=2, rho=0.5, steps=100, rtol=1e-10,
                            geometry="deformed", init="grf", seed=2000),
}


def make_geometry(dim, n, p, geometry, seed=None):
    if geometry == "identity":
        return identity_ctrl(n, p, dim)
    if geometry == "deformed":
        return deformed_cube_ctrl(n, p, dim=dim)
    if geometry == "random":
        return smooth_random_ctrl(n, p, seed, dim=dim)
    raise ValueError(geometry)


def make_initial(dim, n, p, init, seed=0):
    if init == "standing_wave":
        return standing_wave_u0(n, p)
    if init == "grf":
        return grf(n, p, seed, dim=dim)
    raise ValueError(init)


GNET_LAYERS = ((4, 32), (32, 32), (32, 1))


def gnet_random_params(seed, scale=1.0):
    """Seeded parameters of the learned-guess net (tap-major layout, 32,033
    values): He-scaled normal weights, small normal biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in GNET_LAYERS:
        parts.append(rng.standard_normal(27 * ci * co) * scale * np.sqrt(2.0 / (27 * ci)))
        parts.append(rng.standard_normal(co) * 0.05 * scale)
    return np.concatenate(parts)


def multipatch_specs(R=12, n_min=16, n_max=96, seed=7):
    """[(n_r, p_r, geometry_seed_r, initial_seed_r)] of the batched workload."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(R):
        n = int(rng.integers(n_min, n_max + 1))
        p = int(rng.integers(2, 5))
        out.append((n, p, seed * 1000 + r, seed * 1000 + 100 + r))
    return out


def brick_ctrl(P, n, p, r, amp=0.05):
    """Control points [N_dof][3] of patch r (boxes numbered x fastest) of a brick
    of P = (P_x, P_y, P_z) boxes over the unit cube."""
    P = tuple(int(v) for v in P)
    b = (r % P[0], (r // P[0]) % P[1], r // (P[0] * P[1]))
    g = _grid([(b[a] + greville(n, p)) / P[a] for a in range(3)])
    out = g.copy()
    s_ = np.sin(np.pi * g)
    for c in range(3):
        out[:, c] = g[:, c] + amp * s_[:, (c + 1) % 3] * s_[:, (c + 2) % 3]
    return out


def brick_grf(P, n, p, seed, ell=0.1):
    """GRF on the global unknowns of a glued brick (interior global coefficients,
    co-lex): per axis the patch Greville points, shared ends merged."""
    axes = []
    for a in range(3):
        gv = greville(n, p)
        pts = np.concatenate([(b + gv[(1 if b else 0):]) / P[a] for b in range(P[a])])
        axes.append(pts[1:-1])
    return grf_on_axes(axes, seed, ell)
