"""The explicit order-2k generalized-alpha scheme (Sec. 3 for k = 2, Sec. 4 for
general k: stage equations ho1, updates ho2, definitions ho3; initial data as
in Sec. 3), for M U'' + C U' + K U = F.

State: L^a for a = -2 .. N, N = 3k-3, with L^{-2} = U, L^{-1} = V, L^0 = A and
L^a the a-th time derivative of A.  Block j = 1..k has base index a_j = 3j-3.

Readings of the paper used here:
* Stage argument of K.  For blocks j < k (alpha_f = 1, Remark in Sec. 4) the
  stiffness acts on the full Taylor predictor of L^{a_j-2} at t_{n+1},
  T_{a_j-2} = sum_{b >= a_j-2} tau^{b-a_j+2}/(b-a_j+2)! L^b_n.  This is what
  the printed amplification matrices (third rows of B and of Lambda_j) encode;
  the printed stage equations show K L^{3j-5}_n instead, which yields a first
  order method.  For block k (alpha_f = 0) K acts on L^{N-2}_n itself.
* Parameters.  The boxed type-j formulas (j < k) are evaluated at
  rho_b = rho_s = -rho; the type-k formulas at rho_b = rho_s = +rho.  With the
  literal sign the characteristic polynomial of Lambda_j at Omega_b does not
  factor as the printed (lambda + rho_b)^2 (lambda + rho_s), and the stability
  interval shrinks for k >= 2, against the paper's claim that it does not
  depend on k.  gamma_j = 1/2 - alpha_fj + alpha_j (Theorem 2).
* The factorial printed as "3(k-j) !" is (3(k-j))!.
* Damping and forcing.  C acts on the predictor one derivative above K's
  argument: T_{a_j-1} for j < k, L^{N-1}_n for j = k; the load derivative
  F^{(a_j)} is taken at t_n + alpha_fj tau (t_{n+1} for j < k, t_n for j = k).
* Initial data for general k (printed for k = 2 only): L^{-2} = U_0,
  L^{-1} = V_0, L^a = M^{-1}(F^{(a)}(0) - C L^{a-1} - K L^{a-2}) for a = 0..N.
"""
from math import factorial

import numpy as np


# ---- boxed parameter formulas of Sec. 4, as printed ------------------------

def printed_type_j(rb, rs):
    """(alpha, beta, Omega_b, Omega_s) of a block j < k, as printed."""
    alpha = (2 - (1 + rb) * rs) / ((-1 + rb) * (-1 + rs))
    beta = ((1 + rb) * (-1 + rb * rs) ** 2
            / ((-1 + rb) ** 2 * (-1 + rs) * (-2 + rs + rb * rs)))
    omega_b = 2 - 2 * rb - rs + rs * rb ** 2
    omega_s = (4 * (1 - rb) * (2 - rb * rs - rs) * (3 + rb - rs - 3 * rb * rs)
               / (2 * (5 - rb ** 2) + (5 - 13 * rb - rb ** 2 - rb ** 3) * rs
                  - (1 + rb) ** 3 * rs ** 2))
    return alpha, beta, omega_b, omega_s


def printed_type_k(rb, rs):
    """(alpha, beta, Omega_b, Omega_s) of the last block k, as printed."""
    alpha = (2 + (1 - rb) * rs) / ((1 + rb) * (1 + rs))
    beta = ((-5 - 3 * rb - 4 * rs + 2 * rb * rs + 2 * rb ** 2 * rs - rs ** 2 + rb * rs ** 2)
            / ((1 + rb) ** 2 * (-2 - 3 * rs + rb * rs - rs ** 2 + rb * rs ** 2)))
    omega_b = 2 + 2 * rb + rs - rs * rb ** 2
    omega_s = (4 * (1 + rb) * (2 - rb * rs + rs) * (3 - rb + rs - 3 * rb * rs)
               / (2 * (5 - rb ** 2) + (5 - 13 * rb - rb ** 2 + rb ** 3) * rs
                  - (1 - rb) ** 3 * rs ** 2))
    return alpha, beta, omega_b, omega_s


def block_params(k, rho, rho_s=None):
    """[(alpha_j, beta_j, gamma_j, alpha_fj)] for j = 1..k (readings above).
    rho is rho_b; rho_s (default rho_b) gives the two-parameter family
    rho_s <= rho_b of the Remark in Sec. 3 (type-j formulas at (-rho_b, -rho_s),
    type-k at (rho_b, rho_s))."""
    rs = rho if rho_s is None else rho_s
    out = []
    for j in range(1, k + 1):
        if j < k:
            a, b, _, _ = printed_type_j(-rho, -rs)
            af = 1.0
        else:
            a, b, _, _ = printed_type_k(rho, rs)
            af = 0.0
        out.append((a, b, 0.5 - af + a, af))
    return out


# ---- one step ---------------------------------------------------------------

def predictors(L, tau, k):
    """T_a = sum_{b=a..N} tau^{b-a}/(b-a)! L^b for a = -2..N (the Taylor parts
    of the updates ho2 and of P_{n,j}, A_n^{alpha_j} in ho3)."""
    N = 3 * k - 3
    return {a: sum(tau ** (b - a) / factorial(b - a) * L[b] for b in range(a, N + 1))
            for a in range(-2, N + 1)}


def stage_arguments(L, T, k):
    """Argument Y_j of K in stage equation j (reading above)."""
    N = 3 * k - 3
    return [T[3 * j - 5] if j < k else L[N - 2] for j in range(1, k + 1)]


def update(L, T, X, tau, k, rho, rho_s=None):
    """New state from the stage solutions X_j = L^{a_j}(A_n)^{alpha_j}:
    P_{n,j} from ho3 (X_j = T_{a_j} + alpha_j P_{n,j}), then ho2."""
    new = {}
    for j, (al, be, ga, _) in enumerate(block_params(k, rho, rho_s), start=1):
        a = 3 * j - 3
        P = (X[j - 1] - T[a]) / al
        new[a] = T[a] + P
        new[a - 1] = T[a - 1] + ga * tau * P
        new[a - 2] = T[a - 2] + be * tau ** 2 * P
    return new


def damping_arguments(L, T, k):
    """Argument Z_j of C in stage equation j, by the reading used for K: the
    full Taylor predictor T_{a_j-1} for j < k, L^{N-1}_n for j = k."""
    N = 3 * k - 3
    return [T[3 * j - 4] if j < k else L[N - 1] for j in range(1, k + 1)]


def stage_times(t, tau, k, rho):
    """Times t_n + alpha_fj tau at which stage j evaluates its forcing."""
    return [t + af * tau for (_, _, _, af) in block_params(k, rho)]


def step(L, tau, k, rho, apply_K, solve_M, apply_C=None, forcing=None, t=0.0, rho_s=None):
    """One time step from t_n = t: predictors, the k stage solves
    M X_j = F^{(a_j)}(t_n + alpha_fj tau) - C Z_j - K Y_j (eq. ho1), and the
    3k-vector update.  apply_C (damping) and forcing(a, t) (the a-th time
    derivative of the load vector) may be None."""
    T = predictors(L, tau, k)
    Y = stage_arguments(L, T, k)
    b = [-apply_K(y) for y in Y]
    if apply_C is not None:
        b = [bj - apply_C(z) for bj, z in zip(b, damping_arguments(L, T, k))]
    if forcing is not None:
        ts = stage_times(t, tau, k, rho)
        b = [bj + forcing(3 * j, ts[j]) for j, bj in enumerate(b)]
    X = [solve_M(bj) for bj in b]
    return update(L, T, X, tau, k, rho, rho_s)


def initial_state(U0, V0, k, apply_K, solve_M, apply_C=None, forcing=None):
    """L^{-2} = U0, L^{-1} = V0, L^a = M^{-1}(F^{(a)}(0) - C L^{a-1} - K L^{a-2}),
    a = 0..N (the initial solves of Sec. 3, continued to general k)."""
    N = 3 * k - 3
    L = {-2: np.asarray(U0, dtype=np.float64), -1: np.asarray(V0, dtype=np.float64)}
    for a in range(0, N + 1):
        r = -apply_K(L[a - 2])
        if apply_C is not None:
            r = r - apply_C(L[a - 1])
        if forcing is not None:
            r = r + forcing(a, 0.0)
        L[a] = solve_M(r)
    return L


# ---- scalar test equation x'' = -lambda x -----------------------------------

def amplification_matrix(k, rho, theta, rho_s=None):
    """G with U_{n+1} = G U_n for the scaled scalar state
    [U, tau V, tau^2 A, tau^3 L^1, ...] (tau = 1, lambda = Theta), obtained by
    running ``step`` on unit vectors."""
    N = 3 * k - 3
    idx = list(range(-2, N + 1))
    G = np.zeros((len(idx), len(idx)))
    for c, a in enumerate(idx):
        L = {b: np.float64(1.0 if b == a else 0.0) for b in idx}
        new = step(L, 1.0, k, rho, lambda y: theta * y, lambda b: b, rho_s=rho_s)
        for r, b in enumerate(idx):
            G[r, c] = new[b]
    return G


def spectral_radius(k, rho, theta, rho_s=None):
    return float(np.max(np.abs(np.linalg.eigvals(amplification_matrix(k, rho, theta, rho_s)))))


def stability_limit(k, rho, hi=8.0, tol=1e-10, rho_s=None):
    """Largest Theta = tau^2 lambda up to which the spectral radius stays <= 1
    (scan, then bisection on the first crossing)."""
    grid = np.linspace(1e-3, hi, 4001)
    prev = grid[0]
    for th in grid:
        if spectral_radius(k, rho, th, rho_s) > 1 + 1e-9:
            lo, up = prev, th
            while up - lo > tol:
                mid = 0.5 * (lo + up)
                if spectral_radius(k, rho, mid, rho_s) > 1 + 1e-9:
                    up = mid
                else:
                    lo = mid
            return lo
        prev = th
    return float("inf")
