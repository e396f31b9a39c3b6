// C ABI of the library: patch setup, operator applies, preconditioner, PCG
// mass solves and the order-2k generalized-alpha time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"

namespace ga {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

}  // namespace ga

using namespace ga;

namespace ga {

// Stability limit: the lambda = -1 crossing of the characteristic polynomial
// of the last diagonal block (printed in Sec. 3), i.e. Theta (8 beta - 4 gamma)
// = 16 alpha - 8, with the block-k parameters.
// block k: the printed type-k formulas at (rho_b, rho_s)
void block_k_params2(double rho_b, double rho_s, double& a, double& b, double& g) {
  const double rb = rho_b, rs = rho_s;
  a = (2 + (1 - rb) * rs) / ((1 + rb) * (1 + rs));
  b = (-5 - 3 * rb - 4 * rs + 2 * rb * rs + 2 * rb * rb * rs - rs * rs + rb * rs * rs) /
      ((1 + rb) * (1 + rb) * (-2 - 3 * rs + rb * rs - rs * rs + rb * rs * rs));
  g = 0.5 + a;  // gamma = 1/2 - alpha_f + alpha with alpha_f = 0
}

// blocks j < k: the printed type-j formulas evaluated at (-rho_b, -rho_s)
void block_j_params2(double rho_b, double rho_s, double& a, double& b, double& g) {
  const double rb = -rho_b, rs = -rho_s;
  a = (2 - (1 + rb) * rs) / ((-1 + rb) * (-1 + rs));
  b = (1 + rb) * (-1 + rb * rs) * (-1 + rb * rs) /
      ((-1 + rb) * (-1 + rb) * (-1 + rs) * (-2 + rs + rb * rs));
  g = 0.5 - 1.0 + a;  // alpha_f = 1
}

void block_k_params(double rho, double& a, double& b, double& g) { block_k_params2(rho, rho, a, b, g); }
void block_j_params(double rho, double& a, double& b, double& g) { block_j_params2(rho, rho, a, b, g); }

}  // namespace ga

namespace {

template <class T>
int upload(T** dst, const std::vector<T>& v) {
  int rc = dalloc((void**)dst, v.size() * sizeof(T));
  if (rc) return rc;
  GA_TRY_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return GA_OK;
}


// ---- optional HIP-event timing of the operator and preconditioner launches ----
struct ProfState {
  unsigned kinds = 0;  // bit k set: launches of kind k are timed
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[4];
  double total_ms[4] = {0, 0, 0, 0};
  long long count[4] = {0, 0, 0, 0};
};
ProfState g_prof;

hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_drain(int kind) {
  for (auto& pr : g_prof.pending[kind]) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess &&
        hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      g_prof.total_ms[kind] += ms;
      g_prof.count[kind] += 1;
    }
    g_prof.pool.push_back(pr.first);
    g_prof.pool.push_back(pr.second);
  }
  g_prof.pending[kind].clear();
}

struct ProfScope {
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int k, hipStream_t s) : kind(k), st(s) {
    if (!((g_prof.kinds >> kind) & 1u)) return;
    if (g_prof.pending[kind].size() > 4096) prof_drain(kind);
    a = prof_event();
    b = prof_event();
    if (a && b) hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a || !b) return;
    hipEventRecord(b, st);
    g_prof.pending[kind].push_back({a, b});
  }
};

// grow the patch work area to hold `nvec` vectors of n_free doubles
int ensure_work(ga_patch* pt, int nvec) {
  size_t need = (size_t)nvec * (size_t)pt->n_free * sizeof(double);
  if (need <= pt->work_bytes) return GA_OK;
  if (pt->work) hipFree(pt->work);
  pt->work = nullptr;
  pt->work_bytes = 0;
  int rc = dalloc((void**)&pt->work, need);
  if (rc) return rc;
  pt->work_bytes = need;
  return GA_OK;
}

constexpr int MAX_NR = 3;  // right-hand sides per kernel pass
int ensure_packed(ga_patch* pt, int prec, hipStream_t st);

int op_apply(ga_patch* pt, int mode, int nr, double alpha, const double* x, double* y,
             hipStream_t st, const double* gate = nullptr) {
  // y += alpha * Op x, in chunks of at most op3d_max_nr right-hand sides; with a gate
  // (NSCAL scalars per right-hand side) right-hand sides whose S_ACTIVE is 0 are skipped
  const int cmax = pt->dim == 3 ? op3d_max_nr(pt->p, mode) : MAX_NR;
  for (int r0 = 0; r0 < nr; r0 += cmax) {
    int c = nr - r0 < cmax ? nr - r0 : cmax;
    const double* xc = x ? x + (size_t)r0 * pt->n_free : nullptr;
    double* yc = y + (size_t)r0 * pt->n_free;
    const double* gc = gate ? gate + (size_t)r0 * NSCAL : nullptr;
    ProfScope prof(mode == 1 ? 1 : 0, st);
    int rc = pt->dim == 3 ? launch_op3d(mode, c, pt, xc, yc, alpha, st, gc)
                          : launch_op2d(mode, c, pt, xc, yc, alpha, st, gc);
    if (check_launch(rc, "operator")) return GA_EDEVICE;
  }
  return GA_OK;
}

// z = P^{-1} r using two scratch vectors t0, t1 (each nr * n_free): one dense
// contraction per axis, the scaling folded into the first and last pass
// (generic GEMM passes for axes longer than 256)
int pinv_apply(ga_patch* pt, int nr, const double* r, double* z, double* t0, double* t1,
               hipStream_t st) {
  const size_t n = pt->n_free;
  const int m0 = pt->mf[0], m1 = pt->mf[1], m2 = pt->mf[2];
  ProfScope prof(2, st);
  if (pt->pinv_mode == GA_PINV_MFMA) {
    int rc = ensure_packed(pt, GA_FP64, st);
    if (rc) return rc;
    const void* apk[3] = {pt->apk[GA_FP64][0], pt->apk[GA_FP64][1], pt->apk[GA_FP64][2]};
    return check_launch(launch_pinv_mfma_f64(pt->dim, pt->mf, nr, r, z, t0, t1, apk, pt->s,
                                             (long long)n, st),
                        "matrix-core preconditioner");
  }
  if (pt->pinv_mode != GA_PINV_DENSE) {
    const double* cb[3] = {pt->cb[0], pt->cb[1], pt->cb[2]};
    const int rc = launch_pinv_band<double>(pt->dim, pt->p, pt->mf, nr, r, z, t0, t1, cb, pt->s,
                                            (long long)n, st);
    if (rc == 0) return check_launch(0, "preconditioner");
    if (rc < 0) return check_launch(-1, "preconditioner");
  }
  const bool fast = pinv_axis_supported(m0) && pinv_axis_supported(m1) &&
                    (pt->dim == 2 || pinv_axis_supported(m2));
  if (fast) {
    launch_pinv_contig<double>(r, t1, pt->Minv[0], m0, (long long)nr * m1 * m2, (long long)m1 * m2,
                       (long long)n, pt->s, nullptr, st);
    if (pt->dim == 2) {
      launch_pinv_strided<double>(t1, z, pt->Minv[1], m1, m0, m0, 0, 1, (long long)n, nr, nullptr,
                          pt->s, st);
    } else {
      launch_pinv_strided<double>(t1, t0, pt->Minv[1], m1, m0, m0, (long long)m0 * m1, m2, (long long)n,
                          nr, nullptr, nullptr, st);
      launch_pinv_strided<double>(t0, z, pt->Minv[2], m2, (long long)m0 * m1, (long long)m0 * m1, 0, 1,
                          (long long)n, nr, nullptr, pt->s, st);
    }
    return check_launch(0, "preconditioner");
  }
  launch_scale_mul(t0, r, pt->s, nr, n, st);
  // x axis: rows of length m0:  t1[row][i] = sum_j t0[row][j] Ax[j][i]  (Ax symmetric)
  launch_gemm((int)((size_t)nr * m1 * m2), m0, m0, t0, m0, 0, pt->Minv[0], m0, 0, t1, m0, 0, 1, st);
  // y axis: per (r, z) plane: t0[i][x] = sum_j Ay[i][j] t1[j][x]
  launch_gemm(m1, m0, m1, pt->Minv[1], m1, 0, t1, m0, (long long)m0 * m1, t0, m0,
              (long long)m0 * m1, nr * m2, st);
  const double* last = t0;
  if (pt->dim == 3) {
    // z axis: per r: t1[i][yx] = sum_j Az[i][j] t0[j][yx]
    launch_gemm(m2, m0 * m1, m2, pt->Minv[2], m2, 0, t0, (long long)m0 * m1, (long long)n, t1,
                (long long)m0 * m1, (long long)n, nr, st);
    last = t1;
  }
  launch_scale_mul(z, last, pt->s, nr, n, st);
  return check_launch(0, "preconditioner");
}

struct SolveBufs {
  double *r, *z, *p, *q, *t0, *t1;
};

// One PCG iteration with device-side control: every launch is gated by the
// per-system flags (a converged system is skipped on the device).  The
// systems the schedule expects to be active at iteration `it` share one mass
// apply; every other system gets a gated launch of its own, which returns at
// once if that system has converged, so the iterates never depend on the
// schedule.
int gated_iteration(ga_patch* pt, int nr, int it, double* x, const SolveBufs& w, hipStream_t st) {
  const size_t n = pt->n_free;
  const double* gate = pt->scal;
  double* partA = pt->red;
  launch_fill_gated(nr, w.q, n, gate, st);
  int a = nr, b = 0;
  for (int r = 0; r < nr; ++r)
    if (pt->hint[r] > it) { a = std::min(a, r); b = r + 1; }
  if (a >= b) { a = 0; b = nr; }
  {
    ProfScope prof(0, st);
    int rc = 0;
    auto mass = [&](int r0, int c) {
      return pt->dim == 3 ? launch_op3d(0, c, pt, w.p + (size_t)r0 * n, w.q + (size_t)r0 * n, 1.0,
                                        st, gate + (size_t)r0 * NSCAL)
                          : launch_op2d(0, c, pt, w.p + (size_t)r0 * n, w.q + (size_t)r0 * n, 1.0,
                                        st, gate + (size_t)r0 * NSCAL);
    };
    for (int r0 = a; r0 < b && !rc; r0 += MAX_NR) rc = mass(r0, std::min(MAX_NR, b - r0));
    for (int r = 0; r < nr && !rc; ++r)
      if (r < a || r >= b) rc = mass(r, 1);
    if (check_launch(rc, "gated mass apply")) return GA_EDEVICE;
  }
  launch_dot_partial(nr, w.p, w.q, n, partA, st, gate);
  launch_cg_alpha(nr, partA, pt->scal, st);
  launch_cg_xr(nr, x, w.r, w.p, w.q, pt->scal, n, st);
  {
    ProfScope prof(2, st);
    const double* cb[3] = {pt->cb[0], pt->cb[1], pt->cb[2]};
    if (launch_pinv_band<double>(pt->dim, pt->p, pt->mf, nr, w.r, w.z, w.t0, w.t1, cb, pt->s,
                                 (long long)n, st, gate) != 0)
      return check_launch(-1, "gated preconditioner");
  }
  launch_dot_partial(nr, w.r, w.z, n, partA, st, gate);
  launch_cg_beta(nr, partA, pt->scal, st);
  launch_cg_p(nr, w.p, w.z, pt->scal, n, st);
  return check_launch(0, "gated pcg iteration");
}

// One single-reduction (Chronopoulos-Gear) PCG iteration under device control, six
// launches: w = M z (gated, grouped by the schedule as in gated_iteration), the
// partial sums of delta = z^T w, one kernel that completes delta in every workgroup,
// takes the alpha/beta step and updates p, s = M p, x and r, and the three
// preconditioner passes, the last of which sums gamma = r^T z (its last workgroup
// per right-hand side completes the sum and applies the stopping test, so a
// converged system skips the next mass apply).
int cgcg_iteration(ga_patch* pt, int nr, int it, double* x, double* r, double* z, double* p,
                   double* sv, double* w, double* t0, double* t1, hipStream_t st) {
  const size_t n = pt->n_free;
  const double* gate = pt->scal;
  int a = nr, b = 0;
  for (int q = 0; q < nr; ++q)
    if (pt->hint[q] > it) { a = std::min(a, q); b = q + 1; }
  if (a >= b) { a = 0; b = nr; }
  {
    ProfScope prof(0, st);
    int rc = 0;
    for (int r0 = a; r0 < b && !rc; r0 += MAX_NR) {
      const int c = std::min(MAX_NR, b - r0);
      rc = launch_op3d(0, c, pt, z + (size_t)r0 * n, w + (size_t)r0 * n, 1.0, st,
                       gate + (size_t)r0 * NSCAL);
    }
    for (int q = 0; q < nr && !rc; ++q)
      if (q < a || q >= b)
        rc = launch_op3d(0, 1, pt, z + (size_t)q * n, w + (size_t)q * n, 1.0, st,
                         gate + (size_t)q * NSCAL);
    if (check_launch(rc, "single-reduction mass apply")) return GA_EDEVICE;
  }
  launch_dot_partial(nr, z, w, n, pt->red, st, gate);
  launch_cgcg_update(nr, it, x, r, p, sv, w, z, pt->red, pt->scal, n, st);
  {
    ProfScope prof(2, st);
    const double* cb[3] = {pt->cb[0], pt->cb[1], pt->cb[2]};
    CgFuse fz{pt->cgf_part, pt->cgf_cnt, pt->scal, CGF_PSTRIDE};
    if (launch_pinv_band_cgcg(pt->p, pt->mf, nr, r, z, t0, t1, cb, pt->s, (long long)n, st, gate, fz))
      return check_launch(-1, "single-reduction preconditioner");
  }
  return check_launch(0, "single-reduction pcg iteration");
}

int ensure_cgf(ga_patch* pt) {
  if (pt->cgf_part) return GA_OK;
  int rc = dalloc((void**)&pt->cgf_part, sizeof(double) * CGF_MAXRHS * CGF_PSTRIDE);
  if (rc) return rc;
  if ((rc = dalloc((void**)&pt->cgf_cnt, sizeof(unsigned) * 64))) return rc;
  GA_TRY_HIP(hipMemset(pt->cgf_cnt, 0, sizeof(unsigned) * 64));
  return GA_OK;
}

// PCG for nr right-hand sides; x holds the guess (zero_guess: ignored and set to 0)
int solve_impl(ga_patch* pt, int nr, const double* b, double* x, double rtol, int maxit,
               bool zero_guess, int* iters_out, double* relres_out, hipStream_t st) {
  const size_t n = pt->n_free;
  const bool fused = pt->cg_ctrl == GA_CG_FUSED && pt->dim == 3 && pt->pinv_mode == GA_PINV_AUTO &&
                     nr <= 16 && pinv_band_fits(3, pt->p, pt->mf, sizeof(double));
  // slots of nr vectors: r, a copy of b, z, q, p, t0 (two), t1 (two), s (fused):
  // with a guess, [r | b] -> [z | q] is one preconditioner apply of 2 nr right-hand
  // sides (its passes take as long for 2 nr as for nr: too few lines for the chip)
  int rc = ensure_work(pt, fused ? 10 * nr : 9 * nr);
  if (rc) return rc;
  if (fused && (rc = ensure_cgf(pt))) return rc;
  SolveBufs w;
  double* base = pt->work;
  const size_t tot = (size_t)nr * n;
  w.r = base;
  double* bq = base + tot;
  w.z = base + 2 * tot;
  w.q = base + 3 * tot;
  w.p = base + 4 * tot;
  w.t0 = base + 5 * tot;
  w.t1 = base + 7 * tot;
  double* partA = pt->red;
  double* partB = pt->red + (size_t)16 * RED_BLOCKS;
  const double* pbn = nullptr;
  if (zero_guess) {
    launch_fill(x, 0.0, tot, st);
    launch_copy(w.r, b, tot, st);
    if ((rc = pinv_apply(pt, nr, w.r, w.z, w.t0, w.t1, st))) return rc;
    launch_dot_partial(nr, w.r, w.z, n, partA, st);
  } else {
    launch_copy(w.r, b, tot, st);
    launch_copy(bq, b, tot, st);
    if ((rc = op_apply(pt, 0, nr, -1.0, x, w.r, st))) return rc;
    if ((rc = pinv_apply(pt, 2 * nr, w.r, w.z, w.t0, w.t1, st))) return rc;
    launch_dot_partial(nr, w.r, w.z, n, partA, st);
    launch_dot_partial(nr, b, w.q, n, partB, st);
    pbn = partB;
  }
  launch_cg_start(nr, partA, pbn, pt->scal, rtol * rtol, st);
  if (!zero_guess) launch_cg_fallback(nr, x, w.r, w.z, b, w.q, pt->scal, n, st);
  if (check_launch(0, "pcg start")) return GA_EDEVICE;
  int it = 0;
  if (fused) {
    // single-reduction PCG: w (in q) starts at zero, s is the last vector
    double* sv = base + 9 * tot;
    launch_fill(w.q, 0.0, tot, st);
    if (pt->hint_nr == nr) {
      int hmax = 0;
      for (int r = 0; r < nr; ++r) hmax = std::max(hmax, pt->hint[r]);
      for (; it < std::min(hmax, maxit); ++it)
        if ((rc = cgcg_iteration(pt, nr, it, x, w.r, w.z, w.p, sv, w.q, w.t0, w.t1, st))) return rc;
      pt->n_spec += it;
    }
    for (;; ++it) {
      GA_TRY_HIP(hipMemcpyAsync(pt->host_scal, pt->scal, sizeof(double) * NSCAL * nr,
                                hipMemcpyDeviceToHost, st));
      GA_TRY_HIP(hipStreamSynchronize(st));
      pt->n_checks += 1;
      bool any = false;
      for (int r = 0; r < nr; ++r) any |= pt->host_scal[r * NSCAL + S_ACTIVE] != 0.0;
      if (!any || it >= maxit) break;
      if ((rc = cgcg_iteration(pt, nr, it, x, w.r, w.z, w.p, sv, w.q, w.t0, w.t1, st))) return rc;
    }
  } else {
  launch_copy(w.p, w.z, tot, st);
  // device-side control: enqueue the iterations the last solve of nr systems
  // needed without reading the flags in between
  const bool dev = pt->cg_ctrl != GA_CG_HOST && pt->pinv_mode == GA_PINV_AUTO && nr <= 16 &&
                   pt->hint_nr == nr && pinv_band_fits(pt->dim, pt->p, pt->mf, sizeof(double));
  if (dev) {
    int hmax = 0;
    for (int r = 0; r < nr; ++r) hmax = std::max(hmax, pt->hint[r]);
    for (; it < std::min(hmax, maxit); ++it)
      if ((rc = gated_iteration(pt, nr, it, x, w, st))) return rc;
    pt->n_spec += it;
  }
  for (;; ++it) {
    GA_TRY_HIP(hipMemcpyAsync(pt->host_scal, pt->scal, sizeof(double) * NSCAL * nr,
                              hipMemcpyDeviceToHost, st));
    GA_TRY_HIP(hipStreamSynchronize(st));
    pt->n_checks += 1;
    // right-hand sides a .. b-1 span the active ones; the operator and the
    // preconditioner skip converged ones outside that range (their step
    // sizes are zero, so their q and z are never used)
    int a = nr, b = 0;
    for (int r = 0; r < nr; ++r)
      if (pt->host_scal[r * NSCAL + S_ACTIVE] != 0.0) { a = std::min(a, r); b = r + 1; }
    if (a >= b || it >= maxit) break;
    const size_t o = (size_t)a * n, cnt = (size_t)(b - a);
    launch_fill(w.q + o, 0.0, cnt * n, st);
    if ((rc = op_apply(pt, 0, (int)cnt, 1.0, w.p + o, w.q + o, st))) return rc;
    launch_dot_partial(nr, w.p, w.q, n, partA, st);
    launch_cg_alpha(nr, partA, pt->scal, st);
    launch_cg_xr(nr, x, w.r, w.p, w.q, pt->scal, n, st);
    if ((rc = pinv_apply(pt, (int)cnt, w.r + o, w.z + o, w.t0, w.t1, st))) return rc;
    launch_dot_partial(nr, w.r, w.z, n, partA, st);
    launch_cg_beta(nr, partA, pt->scal, st);
    launch_cg_p(nr, w.p, w.z, pt->scal, n, st);
    if (check_launch(0, "pcg iteration")) return GA_EDEVICE;
  }
  }
  bool ok = true;
  for (int r = 0; r < nr; ++r) {
    const double* s = pt->host_scal + r * NSCAL;
    pt->n_solves += 1;
    if (!zero_guess) {
      pt->n_guessed += 1;
      pt->n_fallbacks += s[S_FALLBACK] != 0.0 ? 1 : 0;
      pt->guess_rel_sum += s[S_BN2] > 0 ? std::sqrt(std::fabs(s[S_RZ0] / s[S_BN2])) : 0.0;
    }
    if (iters_out) iters_out[r] = (int)s[S_ITERS];
    if (relres_out) relres_out[r] = s[S_BN2] > 0 ? std::sqrt(std::fabs(s[S_RZ] / s[S_BN2])) : 0.0;
    if (s[S_ACTIVE] != 0.0) ok = false;
    if (!std::isfinite(s[S_RZ])) ok = false;
    if (r < 16) pt->hint[r] = (int)s[S_ITERS];
  }
  pt->hint_nr = nr;
  if (!ok) {
    set_error("PCG did not converge within maxit");
    return GA_ENOCONV;
  }
  return GA_OK;
}

// ---- mixed precision: FP32 inner PCG inside an FP64 iterative refinement ----

// FP32 copies of W, the 1-D inverses, the band factors and the scaling (built on
// first use)
int ensure_mixed(ga_patch* pt, hipStream_t st) {
  if (pt->W32) return GA_OK;
  if (pt->dim != 3) { set_error("FP32 and BF16 arithmetic need a 3-D patch"); return GA_EINVAL; }
  int rc;
  if ((rc = dalloc((void**)&pt->W32, pt->nW * sizeof(float))) ||
      (rc = dalloc((void**)&pt->s32, pt->n_free * sizeof(float))))
    return rc;
  launch_to_f32(pt->W32, pt->W, pt->nW, st);
  launch_to_f32(pt->s32, pt->s, pt->n_free, st);
  for (int a = 0; a < 3; ++a) {
    const size_t mm = (size_t)pt->mf[a] * pt->mf[a];
    if ((rc = dalloc((void**)&pt->Minv32[a], mm * sizeof(float)))) return rc;
    launch_to_f32(pt->Minv32[a], pt->Minv[a], mm, st);
    const size_t nc = pt->ax[a].chol.size();
    if ((rc = dalloc((void**)&pt->cb32[a], nc * sizeof(float)))) return rc;
    launch_to_f32(pt->cb32[a], pt->cb[a], nc, st);
  }
  return check_launch(0, "mixed-precision setup");
}

// the low-precision factor copy an operator apply needs (mode 0 W, 1 G), built on
// first use: FP32 (W32, G32) or BF16 (W16, G16), rounded to nearest from FP64
int ensure_factors(ga_patch* pt, int mode, int prec, hipStream_t st) {
  int rc = ensure_mixed(pt, st);
  if (rc) return rc;
  const double* src = mode == 1 ? pt->G : pt->W;
  const size_t cnt = mode == 1 ? pt->nG : pt->nW;
  if (prec == GA_FP32) {
    float** dst = mode == 1 ? &pt->G32 : &pt->W32;
    if (*dst) return GA_OK;
    if ((rc = dalloc((void**)dst, cnt * sizeof(float)))) return rc;
    launch_to_f32(*dst, src, cnt, st);
  } else if (prec == GA_BF16) {
    unsigned short** dst = mode == 1 ? &pt->G16 : &pt->W16;
    if (*dst) return GA_OK;
    if ((rc = dalloc((void**)dst, cnt * sizeof(unsigned short)))) return rc;
    launch_to_bf16(*dst, src, cnt, st);
  } else {
    return GA_OK;
  }
  return check_launch(0, "low-precision factor copy");
}

// the dense 1-D inverses packed for the matrix cores in arithmetic prec (built on
// first use)
int ensure_packed(ga_patch* pt, int prec, hipStream_t st) {
  for (int a = 0; a < pt->dim; ++a) {
    if (pt->apk[prec][a]) continue;
    if (!pinv_mfma_supported(prec, pt->mf[a])) {
      set_error("the matrix-core preconditioner supports axes of at most 256 free coefficients");
      return GA_EINVAL;
    }
    int rc = dalloc(&pt->apk[prec][a], pinv_mfma_pack_bytes(prec, pt->mf[a]));
    if (rc) return rc;
    if (pinv_mfma_pack(prec, pt->Minv[a], pt->mf[a], pt->apk[prec][a], st))
      return check_launch(-1, "packing the 1-D inverses");
  }
  return GA_OK;
}

// z = P^{-1} r with FP32 vectors: GA_FP32 with the patch's preconditioner mode
// (banded FP32 solves, dense FP32 products on the vector ALU, or dense FP32 products
// on the matrix cores), GA_BF16 on the matrix cores with BF16 operands
int pinv_apply_lp(ga_patch* pt, int prec, int nr, const float* r, float* z, float* t0, float* t1,
                  hipStream_t st, const double* gate = nullptr) {
  const size_t n = pt->n_free;
  const int m0 = pt->mf[0], m1 = pt->mf[1], m2 = pt->mf[2];
  if (!(pinv_axis_supported(m0) && pinv_axis_supported(m1) && pinv_axis_supported(m2))) {
    set_error("FP32 and BF16 arithmetic support axes of at most 256 free coefficients");
    return GA_EINVAL;
  }
  int rc = ensure_mixed(pt, st);
  if (rc) return rc;
  ProfScope prof(2, st);
  if (prec == GA_BF16 || pt->pinv_mode == GA_PINV_MFMA) {
    if ((rc = ensure_packed(pt, prec, st))) return rc;
    const void* apk[3] = {pt->apk[prec][0], pt->apk[prec][1], pt->apk[prec][2]};
    return check_launch(launch_pinv_mfma_f32(prec, 3, pt->mf, nr, r, z, t0, t1, apk, pt->s32,
                                             (long long)n, st),
                        "matrix-core preconditioner");
  }
  if (pt->pinv_mode != GA_PINV_DENSE) {
    const float* cb[3] = {pt->cb32[0], pt->cb32[1], pt->cb32[2]};
    rc = launch_pinv_band<float>(3, pt->p, pt->mf, nr, r, z, t0, t1, cb, pt->s32, (long long)n, st,
                                 gate);
    if (rc == 0) return check_launch(0, "FP32 preconditioner");
    if (rc < 0) return check_launch(-1, "FP32 preconditioner");
  }
  launch_pinv_contig<float>(r, t1, pt->Minv32[0], m0, (long long)nr * m1 * m2,
                            (long long)m1 * m2, (long long)n, pt->s32, nullptr, st);
  launch_pinv_strided<float>(t1, t0, pt->Minv32[1], m1, m0, m0, (long long)m0 * m1, m2,
                             (long long)n, nr, nullptr, nullptr, st);
  launch_pinv_strided<float>(t0, z, pt->Minv32[2], m2, (long long)m0 * m1, (long long)m0 * m1, 0,
                             1, (long long)n, nr, nullptr, pt->s32, st);
  return check_launch(0, "FP32 preconditioner");
}

// y += alpha Op x with FP32 vectors, FP32 (prec GA_FP32) or BF16 (GA_BF16) factors
int op_apply_lp(ga_patch* pt, int mode, int prec, int nr, float alpha, const float* x, float* y,
                hipStream_t st, const double* gate = nullptr) {
  int rc = ensure_factors(pt, mode, prec, st);
  if (rc) return rc;
  const int cmax = op3d_max_nr(pt->p, mode);
  for (int r0 = 0; r0 < nr; r0 += cmax) {
    const int c = nr - r0 < cmax ? nr - r0 : cmax;
    ProfScope prof(mode == 1 ? 1 : 0, st);
    rc = launch_op3d_lowp(mode, c, pt, x + (size_t)r0 * pt->n_free, y + (size_t)r0 * pt->n_free,
                          alpha, prec, st, gate ? gate + (size_t)r0 * NSCAL : nullptr);
    if (check_launch(rc, "low-precision operator apply")) return GA_EDEVICE;
  }
  return GA_OK;
}

int mass_apply_lp(ga_patch* pt, int prec, int nr, const float* x, float* y, hipStream_t st,
                  const double* gate = nullptr) {
  launch_fill_f32(y, (size_t)nr * pt->n_free, st);
  return op_apply_lp(pt, 0, prec, nr, 1.0f, x, y, st, gate);
}

int read_scalars(ga_patch* pt, int nr, hipStream_t st) {
  GA_TRY_HIP(hipMemcpyAsync(pt->host_scal, pt->scal, sizeof(double) * NSCAL * nr,
                            hipMemcpyDeviceToHost, st));
  GA_TRY_HIP(hipStreamSynchronize(st));
  return GA_OK;
}

// Mixed precision: FP64 iterative refinement around an inner flexible PCG in FP32
// (or with BF16 factors and preconditioner).  Outer pass: the FP64 residual
// r = b - M x (FP64 factors and arithmetic), z = P^{-1} r in the inner precision,
// the outer test sqrt(r^T z) <= rtol sqrt(b^T P^{-1} b) with FP64-accumulated dots;
// the inner PCG for M d = r starts from d = 0 and stops when its residual has
// dropped to max(rtol_remaining / 2, floor) (rtol_remaining = rtol |b|_P / |r|_P, so
// a single pass reaches rtol where the inner precision allows it; floor: what the
// inner arithmetic resolves); then x += d in FP64.  Control stays on the device:
// every inner launch is gated by the per-system inner flags, the host enqueues the
// number of inner iterations the previous solve needed and reads the flags once per
// outer pass.
constexpr int MX_ITERS_LAST = 10;   // outer scalar slots: inner iterations of the last pass,
constexpr int MX_CUT = 11;          //   and whether that pass ended with its inner PCG still active

int solve_mixed_impl(ga_patch* pt, int prec, int nr, const double* b, double* x, double rtol,
                     int maxit, bool zero_guess, int* iters_out, double* relres_out,
                     hipStream_t st) {
  const size_t n = pt->n_free;
  const size_t tot = (size_t)nr * n;
  int rc = ensure_mixed(pt, st);
  if (rc) return rc;
  // r64 and nine FP32 vectors: r, q (b), z, p (P^-1 b), d, t0 (two), t1 (two); with a
  // guess, [r | b] -> [z | P^-1 b] is one preconditioner apply of 2 nr right-hand sides
  if ((rc = ensure_work(pt, 6 * nr))) return rc;
  double* r64 = pt->work;
  float* f = reinterpret_cast<float*>(pt->work + tot);
  float *r32 = f, *q32 = f + tot, *z32 = f + 2 * tot, *p32 = f + 3 * tot, *d32 = f + 4 * tot,
        *t0 = f + 5 * tot, *t1 = f + 7 * tot;
  double* partA = pt->red;
  double* partB = pt->red + (size_t)16 * RED_BLOCKS;
  double* so = pt->scal;                       // outer (FP64 refinement) scalars
  double* si = pt->scal + (size_t)32 * NSCAL;  // inner PCG scalars
  const double floor = prec == GA_BF16 ? 2e-3 : 3e-7;
  // the inner result can be accepted without an FP64 residual only where the FP32 or
  // BF16 rounding (about floor times the residual) is far below the tolerance
  const bool accept = 8.0 * floor <= rtol;
  const int h = prec == GA_BF16 ? 1 : 0;
  int& hint = pt->mx_hint[h];
  if (hint < 1) hint = 2;
  // residual of the initial guess, z = P^{-1} r, and (for a guess) P^{-1} b
  if (zero_guess) {
    launch_fill(x, 0.0, tot, st);
    launch_copy(r64, b, tot, st);
    launch_to_f32(r32, r64, tot, st);
    if ((rc = pinv_apply_lp(pt, prec, nr, r32, z32, t0, t1, st))) return rc;
  } else {
    launch_copy(r64, b, tot, st);
    if ((rc = op_apply(pt, 0, nr, -1.0, x, r64, st))) return rc;
    launch_to_f32(r32, r64, tot, st);
    launch_to_f32(q32, b, tot, st);
    if ((rc = pinv_apply_lp(pt, prec, 2 * nr, r32, z32, t0, t1, st))) return rc;
    launch_dot_ff(nr, q32, p32, n, partB, st);
  }
  launch_dot_ff(nr, r32, z32, n, partA, st);
  launch_mx_outer(nr, partA, zero_guess ? nullptr : partB, so, si, rtol * rtol, floor * floor, 0,
                  st);
  // a guess worse than zero: x = 0, r = b, z = P^{-1} b (q32, p32 hold b and P^{-1} b)
  if (!zero_guess) launch_mx_fallback(nr, x, r64, r32, z32, b, q32, p32, so, n, st);
  bool conv = false;
  int inner_total_max = 0;
  for (int pass = 0; pass < 50; ++pass) {
    if (pass > 0) {
      GA_TRY_HIP(hipMemcpyAsync(pt->host_scal, so, sizeof(double) * NSCAL * 32,
                                hipMemcpyDeviceToHost, st));
      GA_TRY_HIP(hipStreamSynchronize(st));
      pt->n_checks += 1;
      bool any = false, cut = false;
      int its = 0;
      for (int r = 0; r < nr; ++r) {
        const double* s = pt->host_scal + r * NSCAL;
        any |= s[S_ACTIVE] != 0.0;
        cut |= s[MX_CUT] != 0.0;
        its = std::max(its, (int)s[MX_ITERS_LAST]);
        inner_total_max = std::max(inner_total_max, (int)s[S_ITERS]);
      }
      // next solve: as many inner iterations as this pass needed (one more if it was cut short)
      hint = std::min(20, cut ? hint + 1 : std::max(1, its));
      if (!any) { conv = true; break; }
      if (inner_total_max >= maxit) break;
    }
    // inner flexible PCG for M d = r from d = 0 (z32 = P^{-1} r32), gated by the inner flags
    launch_fill_f32(d32, tot, st);
    launch_copy_f32(p32, z32, tot, st);
    for (int it = 0; it < hint; ++it) {
      if ((rc = mass_apply_lp(pt, prec, nr, p32, q32, st, si))) return rc;
      launch_dot_ff(nr, p32, q32, n, partA, st);
      launch_cg_alpha(nr, partA, si, st);
      launch_cg_xr_f32(nr, d32, r32, p32, q32, si, n, st);
      if ((rc = pinv_apply_lp(pt, prec, nr, r32, z32, t0, t1, st, si))) return rc;
      launch_dot2_f32(nr, r32, z32, q32, n, partA, partB, st);
      launch_cg_beta_flex(nr, partA, partB, si, st);
      launch_cg_p_f32(nr, p32, z32, si, n, st);
    }
    if (check_launch(0, "inner PCG")) return GA_EDEVICE;
    // x += d; the systems the inner arithmetic resolves are accepted without an FP64
    // residual; for the others r = b - M x in FP64, z = P^{-1} r, the outer test and
    // the next inner start (the residual launches skip accepted systems)
    launch_add_f32(x, d32, tot, st);
    if (accept) launch_mx_accept(nr, so, si, floor * floor, st);
    launch_copy(r64, b, tot, st);
    if ((rc = op_apply(pt, 0, nr, -1.0, x, r64, st, so))) return rc;
    launch_to_f32(r32, r64, tot, st);
    if ((rc = pinv_apply_lp(pt, prec, nr, r32, z32, t0, t1, st, so))) return rc;
    launch_dot_ff(nr, r32, z32, n, partA, st);
    launch_mx_outer(nr, partA, nullptr, so, si, rtol * rtol, floor * floor, 1, st);
  }
  if (check_launch(0, "mixed-precision solve")) return GA_EDEVICE;
  pt->n_solves += nr;
  for (int r = 0; r < nr; ++r) {
    const double* s = pt->host_scal + r * NSCAL;
    if (!zero_guess) {
      pt->n_guessed += 1;
      pt->n_fallbacks += s[S_FALLBACK] != 0.0 ? 1 : 0;
      pt->guess_rel_sum += s[S_BN2] > 0 ? std::sqrt(std::fabs(s[S_RZ0] / s[S_BN2])) : 0.0;
    }
    if (iters_out) iters_out[r] = (int)s[S_ITERS];
    if (relres_out) relres_out[r] = s[S_BN2] > 0 ? std::sqrt(std::fabs(s[S_RZ] / s[S_BN2])) : 0.0;
    if (!std::isfinite(s[S_RZ])) conv = false;
  }
  if (!conv) {
    set_error("mixed-precision solve did not converge within maxit");
    return GA_ENOCONV;
  }
  return GA_OK;
}

int solve_any(ga_patch* pt, int nr, const double* b, double* x, double rtol, int maxit, int prec,
              bool zero_guess, int* iters_out, double* relres_out, hipStream_t st) {
  if (prec == GA_FP32 || prec == GA_BF16)
    return solve_mixed_impl(pt, prec, nr, b, x, rtol, maxit, zero_guess, iters_out, relres_out, st);
  return solve_impl(pt, nr, b, x, rtol, maxit, zero_guess, iters_out, relres_out, st);
}

}  // namespace

int ga::mixed_setup(ga_patch* pt, hipStream_t st) { return ensure_mixed(pt, st); }

// P^{-1} in FP64 with caller-provided scratch t0, t1 (each nr * n_free); allocates
// nothing as long as the patch's preconditioner data exist (a matrix-core mode
// whose packed inverses are not built yet is refused)
int ga::pinv_apply_scratch(ga_patch* pt, int nr, const double* r, double* z, double* t0, double* t1,
                           hipStream_t st) {
  if (pt->pinv_mode == GA_PINV_MFMA)
    for (int a = 0; a < pt->dim; ++a)
      if (!pt->apk[GA_FP64][a]) {
        set_error("the matrix-core preconditioner data are built by a first ga_apply_Pinv call");
        return GA_EINVAL;
      }
  return pinv_apply(pt, nr, r, z, t0, t1, st);
}

extern "C" {

const char* ga_last_error(void) { return g_err.c_str(); }

int ga_profile(int kinds) {
  if (kinds < 0 || kinds > GA_PROF_ALL) { set_error("ga_profile: kinds must be a mask in [0, 15]"); return GA_EINVAL; }
  for (int k = 0; k < 4; ++k) prof_drain(k);
  for (int k = 0; k < 4; ++k) { g_prof.total_ms[k] = 0.0; g_prof.count[k] = 0; }
  g_prof.kinds = (unsigned)kinds;
  return GA_OK;
}

int ga_profile_query(int kind, double* total_ms, long long* launches) {
  if (kind < 0 || kind > 3 || !total_ms || !launches) { set_error("bad argument"); return GA_EINVAL; }
  prof_drain(kind);
  *total_ms = g_prof.total_ms[kind];
  *launches = g_prof.count[kind];
  return GA_OK;
}

double ga_stability_limit(double rho) {
  double a, b, g;
  block_k_params(rho, a, b, g);
  return (16.0 * a - 8.0) / (8.0 * b - 4.0 * g);
}

int ga_setup_patch(int dim, const int* n_el, int p, const double* ctrl_host, void* stream,
                   ga_patch** out) {
  return ga_setup_patch_ex(dim, n_el, p, ctrl_host, dim == 3 ? 0x3Fu : 0xFu, stream, out);
}

int ga_setup_patch_ex(int dim, const int* n_el, int p, const double* ctrl_host,
                      unsigned dirichlet_faces, void* stream, ga_patch** out) {
  if (!out || !n_el || !ctrl_host) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  if (dim != 2 && dim != 3) { set_error("dim must be 2 or 3"); return GA_EINVAL; }
  if (p < 1 || p > 4) { set_error("p must be in 1..4"); return GA_EINVAL; }
  if (dim == 2 && dirichlet_faces != 0xFu) {
    set_error("2-D patches carry Dirichlet data on all four sides");
    return GA_EINVAL;
  }
  if (dirichlet_faces >> (2 * dim)) { set_error("bad face mask"); return GA_EINVAL; }
  for (int a = 0; a < dim; ++a)
    if (n_el[a] < 1 || n_el[a] > 4096) { set_error("n_el out of range"); return GA_EINVAL; }
  int lo[3] = {1, 1, 1}, mfa[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) {
    lo[a] = (dirichlet_faces >> (2 * a)) & 1u ? 1 : 0;
    const int hi = n_el[a] + p - ((dirichlet_faces >> (2 * a + 1)) & 1u ? 1 : 0);
    mfa[a] = hi - lo[a];
    if (mfa[a] < 1) { set_error("no free coefficients"); return GA_EINVAL; }
  }
  hipStream_t st = S(stream);
  ga_patch* pt = new ga_patch();
  pt->dim = dim;
  pt->p = p;
  long long ndof = 1;
  pt->n_free = 1;
  pt->n_tiles = 1;
  for (int a = 0; a < dim; ++a) {
    pt->n[a] = n_el[a];
    pt->m[a] = n_el[a] + p;
    pt->mf[a] = mfa[a];
    pt->lo[a] = lo[a];
    ndof *= pt->m[a];
    pt->n_free *= pt->mf[a];
  }
  pt->n_quad = 1;
  for (int a = 0; a < dim; ++a) pt->n_quad *= (long long)n_el[a] * (p + 1);
  // element padding of the univariate tables: whole tiles of every layout
  int npad_el[3] = {1, 1, 1};
  if (dim == 3) {
    const int tk = te3_stiff(p), tm = te3_mass(p), q = p + 1;
    for (int a = 0; a < 2; ++a) {
      pt->ntk[a] = (n_el[a] + tk - 1) / tk;
      pt->ntm[a] = (n_el[a] + tm - 1) / tm;
      npad_el[a] = std::max(pt->ntk[a] * tk, pt->ntm[a] * tm);
    }
    npad_el[2] = n_el[2];
    const size_t qz = (size_t)n_el[2] * q;
    pt->nW = (size_t)pt->ntm[0] * pt->ntm[1] * (tm * q) * (tm * q) * qz;
    pt->nG = (size_t)pt->ntk[0] * pt->ntk[1] * (tk * q) * (tk * q) * qz * 6;
  } else {
    const int q = p + 1;
    for (int a = 0; a < 2; ++a) {
      pt->nt[a] = (n_el[a] + TE2 - 1) / TE2;
      npad_el[a] = pt->nt[a] * TE2;
      pt->n_tiles *= pt->nt[a];
    }
    pt->qp_per_tile = (long long)(TE2 * q) * (TE2 * q);
    pt->nW = (size_t)pt->n_tiles * pt->qp_per_tile;
    pt->nG = pt->nW * 3;
  }
  int rc = GA_OK;
  auto fail = [&](int code) { ga_destroy_patch(pt); return code; };
  // univariate tables, padded to whole tiles with zeros
  std::vector<double*> wdev(3, nullptr);
  for (int a = 0; a < dim; ++a) {
    pt->ax[a] = build_axis(n_el[a], p, pt->lo[a], pt->mf[a]);
    const Axis1D& ax = pt->ax[a];
    const size_t per_el = (size_t)ax.q * (p + 1);
    const size_t npad = (size_t)npad_el[a];
    std::vector<double> B(npad * per_el, 0.0), D(npad * per_el, 0.0), B2(npad * per_el, 0.0);
    std::vector<double> w(npad * ax.q, 0.0);
    for (size_t i = 0; i < ax.B.size(); ++i) {
      B[i] = ax.B[i];
      D[i] = ax.D[i];
      B2[i] = ax.B[i] * ax.B[i];
    }
    for (size_t i = 0; i < ax.w.size(); ++i) w[i] = ax.w[i];
    if ((rc = upload(&pt->tabB[a], B)) || (rc = upload(&pt->tabD[a], D)) ||
        (rc = upload(&pt->tabB2[a], B2)) || (rc = upload(&pt->Minv[a], ax.Minv)) ||
        (rc = upload(&pt->cb[a], ax.chol)) ||
        (rc = upload(&wdev[a], w))) {
      for (double* d : wdev) if (d) hipFree(d);
      return fail(rc);
    }
  }
  auto free_w = [&]() { for (double*& d : wdev) if (d) { hipFree(d); d = nullptr; } };
  // control points, SoA [dim][ndof]
  std::vector<double> ctrl((size_t)dim * ndof);
  for (long long i = 0; i < ndof; ++i)
    for (int c = 0; c < dim; ++c) ctrl[(size_t)c * ndof + i] = ctrl_host[(size_t)i * dim + c];
  double* dctrl = nullptr;
  int* dbad = nullptr;
  if ((rc = upload(&dctrl, ctrl))) { free_w(); return fail(rc); }
  if ((rc = dalloc((void**)&dbad, sizeof(int)))) { hipFree(dctrl); free_w(); return fail(rc); }
  if ((rc = dalloc((void**)&pt->W, pt->nW * sizeof(double))) ||
      (rc = dalloc((void**)&pt->G, pt->nG * sizeof(double))) ||
      (rc = dalloc((void**)&pt->diagM, pt->n_free * sizeof(double))) ||
      (rc = dalloc((void**)&pt->s, pt->n_free * sizeof(double))) ||
      (rc = dalloc((void**)&pt->red, sizeof(double) * 32 * RED_BLOCKS)) ||
      (rc = dalloc((void**)&pt->scal, sizeof(double) * NSCAL * 64)) ||
      (rc = dalloc((void**)&pt->flags, sizeof(int) * 16))) {
    hipFree(dctrl); hipFree(dbad); free_w();
    return fail(rc);
  }
  if (hipHostMalloc((void**)&pt->host_scal, sizeof(double) * NSCAL * 64) != hipSuccess) {
    hipFree(dctrl); hipFree(dbad); free_w();
    set_error("hipHostMalloc failed");
    return fail(GA_ENOMEM);
  }
  int hbad = 0;
  hipMemsetAsync(dbad, 0, sizeof(int), st);
  hipMemsetAsync(pt->W, 0, pt->nW * sizeof(double), st);  // padding stays zero
  hipMemsetAsync(pt->G, 0, pt->nG * sizeof(double), st);
  const double* wp[3] = {wdev[0], wdev[1], wdev[2]};
  int lrc = dim == 3 ? launch_geo3d(pt, dctrl, wp, dbad, st) : launch_geo2d(pt, dctrl, wp, dbad, st);
  if (check_launch(lrc, "geometry")) { hipFree(dctrl); hipFree(dbad); free_w(); return fail(GA_EDEVICE); }
  hipMemcpyAsync(&hbad, dbad, sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) {
    set_error("geometry setup failed on the device");
    hipFree(dctrl); hipFree(dbad); free_w();
    return fail(GA_EDEVICE);
  }
  hipFree(dctrl);
  hipFree(dbad);
  free_w();
  if (hbad) {
    set_error("det DF <= 0 at a quadrature point (the map must be orientation preserving)");
    return fail(GA_EGEOMETRY);
  }
  // D = diag(M), s = (Dhat / D)^{1/2}
  launch_fill(pt->diagM, 0.0, pt->n_free, st);
  if ((rc = op_apply(pt, 2, 1, 1.0, nullptr, pt->diagM, st))) return fail(rc);
  std::vector<double*> dh(3, nullptr);
  for (int a = 0; a < dim; ++a)
    if ((rc = upload(&dh[a], pt->ax[a].dhat))) {
      for (double* d : dh) if (d) hipFree(d);
      return fail(rc);
    }
  launch_scaling(pt->s, pt->diagM, dh[0], dh[1], dim == 3 ? dh[2] : nullptr, pt->mf[0], pt->mf[1],
                 dim == 3 ? pt->mf[2] : 1, st);
  hipError_t e = hipStreamSynchronize(st);
  for (double* d : dh) if (d) hipFree(d);
  if (e != hipSuccess) { set_error("setup failed on the device"); return fail(GA_EDEVICE); }
  *out = pt;
  return GA_OK;
}

int ga_destroy_patch(ga_patch* pt) {
  if (!pt) return GA_OK;
  for (int a = 0; a < 3; ++a) {
    if (pt->tabB[a]) hipFree(pt->tabB[a]);
    if (pt->tabD[a]) hipFree(pt->tabD[a]);
    if (pt->tabB2[a]) hipFree(pt->tabB2[a]);
    if (pt->Minv[a]) hipFree(pt->Minv[a]);
    if (pt->cb[a]) hipFree(pt->cb[a]);
    if (pt->cb32[a]) hipFree(pt->cb32[a]);
  }
  if (pt->W) hipFree(pt->W);
  if (pt->G) hipFree(pt->G);
  if (pt->W32) hipFree(pt->W32);
  if (pt->G32) hipFree(pt->G32);
  if (pt->W16) hipFree(pt->W16);
  if (pt->G16) hipFree(pt->G16);
  for (int q = 0; q < 3; ++q)
    for (int a = 0; a < 3; ++a)
      if (pt->apk[q][a]) hipFree(pt->apk[q][a]);
  if (pt->s32) hipFree(pt->s32);
  for (int a = 0; a < 3; ++a)
    if (pt->Minv32[a]) hipFree(pt->Minv32[a]);
  if (pt->diagM) hipFree(pt->diagM);
  if (pt->s) hipFree(pt->s);
  if (pt->work) hipFree(pt->work);
  if (pt->red) hipFree(pt->red);
  if (pt->cgf_part) hipFree(pt->cgf_part);
  if (pt->cgf_cnt) hipFree(pt->cgf_cnt);
  if (pt->scal) hipFree(pt->scal);
  if (pt->flags) hipFree(pt->flags);
  if (pt->host_scal) hipHostFree(pt->host_scal);
  delete pt;
  return GA_OK;
}

int ga_solve_stats(ga_patch* pt, long long* solves, long long* guessed, long long* fallbacks,
                   double* mean_guess_relres, int reset) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (solves) *solves = pt->n_solves;
  if (guessed) *guessed = pt->n_guessed;
  if (fallbacks) *fallbacks = pt->n_fallbacks;
  if (mean_guess_relres) *mean_guess_relres = pt->n_guessed ? pt->guess_rel_sum / pt->n_guessed : 0.0;
  if (reset) { pt->n_solves = pt->n_guessed = pt->n_fallbacks = 0; pt->guess_rel_sum = 0.0; }
  return GA_OK;
}

int ga_patch_info(const ga_patch* pt, long long* n_free, long long* n_quad, int* mf) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (n_free) *n_free = pt->n_free;
  if (n_quad) *n_quad = pt->n_quad;
  if (mf) for (int a = 0; a < 3; ++a) mf[a] = a < pt->dim ? pt->mf[a] : 1;
  return GA_OK;
}

int ga_integrator_set_rho(ga_integrator* it, double rho_b, double rho_s) {
  if (!it) { set_error("null integrator"); return GA_EINVAL; }
  if (!(rho_b >= 0.0 && rho_b < 1.0) || !(rho_s >= 0.0 && rho_s <= rho_b)) {
    set_error("need 0 <= rho_s <= rho_b < 1");
    return GA_EINVAL;
  }
  for (int j = 0; j < it->k; ++j) {
    if (j < it->k - 1) block_j_params2(rho_b, rho_s, it->alpha[j], it->beta[j], it->gamma[j]);
    else block_k_params2(rho_b, rho_s, it->alpha[j], it->beta[j], it->gamma[j]);
  }
  it->rho = rho_b;
  return GA_OK;
}

int ga_patch_tune(ga_patch* pt, int nrhs, int reps, double* best_ms, void* stream) {
  if (!pt || nrhs < 1 || nrhs > 3 || reps < 1) { set_error("bad argument"); return GA_EINVAL; }
  if (pt->dim != 3) { set_error("the operator autotuner is for 3-D patches"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = pt->n_free;
  double *x = nullptr, *y = nullptr;
  int rc;
  if ((rc = dalloc((void**)&x, (size_t)nrhs * n * 8))) return rc;
  if ((rc = dalloc((void**)&y, (size_t)nrhs * n * 8))) { hipFree(x); return rc; }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double total = 0.0;
  rc = GA_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("event creation failed");
    rc = GA_EDEVICE;
  }
  launch_fill(x, 1.0, (size_t)nrhs * n, st);
  launch_fill(y, 0.0, (size_t)nrhs * n, st);
  for (int mode = 0; mode < 2 && rc == GA_OK && pt->ze == 0; ++mode) {
    const int nr = std::min(nrhs, op3d_max_nr(pt->p, mode));
    std::vector<int> cand;   // whole columns, then halving down to 4 layers
    for (int ze = pt->n[2];; ze = (ze + 1) / 2) {
      cand.push_back(ze);
      if (ze <= 4) break;
    }
    double best = 1e30;
    int best_ze = 0;
    for (int ze : cand) {
      pt->ze_op[mode] = ze;
      if (launch_op3d(mode, nr, pt, x, y, 1.0, st)) { rc = check_launch(-1, "tuning"); break; }
      hipEventRecord(e0, st);
      for (int i = 0; i < reps; ++i) launch_op3d(mode, nr, pt, x, y, 1.0, st);
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) { rc = check_launch(-1, "tuning"); break; }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; best_ze = ze; }
    }
    pt->ze_op[mode] = best_ze;
    total += best / reps;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(x);
  hipFree(y);
  if (rc) return rc;
  if (best_ms) *best_ms = total;
  return check_launch(0, "tuning");
}

int ga_patch_tuned_layers(const ga_patch* pt, int* ze_mass, int* ze_stiff) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (ze_mass) *ze_mass = op3d_default_ze(0, pt);
  if (ze_stiff) *ze_stiff = op3d_default_ze(1, pt);
  return GA_OK;
}

int ga_patch_set_cg(ga_patch* pt, int mode) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (mode != GA_CG_HOST && mode != GA_CG_DEVICE && mode != GA_CG_FUSED) {
    set_error("bad PCG control mode");
    return GA_EINVAL;
  }
  pt->cg_ctrl = mode;
  return GA_OK;
}

int ga_cg_stats(const ga_patch* pt, long long* spec_iters, long long* host_checks) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (spec_iters) *spec_iters = pt->n_spec;
  if (host_checks) *host_checks = pt->n_checks;
  return GA_OK;
}

int ga_patch_set_pinv(ga_patch* pt, int mode) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (mode != GA_PINV_AUTO && mode != GA_PINV_DENSE && mode != GA_PINV_MFMA) {
    set_error("bad preconditioner mode");
    return GA_EINVAL;
  }
  pt->pinv_mode = mode;
  return GA_OK;
}

int ga_diag_M(ga_patch* pt, double* d, void* stream) {
  if (!pt || !d) { set_error("null argument"); return GA_EINVAL; }
  GA_TRY_HIP(hipMemcpyAsync(d, pt->diagM, pt->n_free * sizeof(double), hipMemcpyDeviceToDevice,
                            S(stream)));
  return GA_OK;
}

int ga_apply_MK(ga_patch* pt, char which, int nrhs, int prec, double alpha, const double* x,
                double* y, void* stream) {
  if (!pt || !x || !y) { set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1) { set_error("nrhs must be >= 1"); return GA_EINVAL; }
  if (which != 'M' && which != 'K') { set_error("which must be 'M' or 'K'"); return GA_EINVAL; }
  if (prec != GA_FP64 && prec != GA_FP32 && prec != GA_BF16) { set_error("bad prec"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const int mode = which == 'M' ? 0 : 1;
  const size_t tot = (size_t)nrhs * pt->n_free;
  if (prec == GA_FP64) {
    launch_fill(y, 0.0, tot, st);
    return op_apply(pt, mode, nrhs, alpha, x, y, st);
  }
  if (pt->dim != 3) { set_error("FP32 and BF16 applies need a 3-D patch"); return GA_EINVAL; }
  int rc = ensure_work(pt, nrhs);   // nrhs * n_free doubles = FP32 x and y
  if (rc) return rc;
  float* x32 = reinterpret_cast<float*>(pt->work);
  float* y32 = x32 + tot;
  launch_to_f32(x32, x, tot, st);
  launch_fill_f32(y32, tot, st);
  if ((rc = op_apply_lp(pt, mode, prec, nrhs, (float)alpha, x32, y32, st))) return rc;
  launch_to_f64(y, y32, tot, st);
  return check_launch(0, "low-precision apply");
}

int ga_apply_Pinv(ga_patch* pt, int nrhs, int prec, const double* r, double* z, void* stream) {
  if (!pt || !r || !z) { set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1) { set_error("nrhs must be >= 1"); return GA_EINVAL; }
  if (prec != GA_FP64 && prec != GA_FP32 && prec != GA_BF16) { set_error("bad prec"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t tot = (size_t)nrhs * pt->n_free;
  if (prec == GA_FP64) {
    int rc = ensure_work(pt, 6 * nrhs);
    if (rc) return rc;
    double* t0 = pt->work + (size_t)4 * tot;
    double* t1 = pt->work + (size_t)5 * tot;
    return pinv_apply(pt, nrhs, r, z, t0, t1, st);
  }
  if (pt->dim != 3) { set_error("FP32 and BF16 applies need a 3-D patch"); return GA_EINVAL; }
  int rc = ensure_work(pt, 2 * nrhs);   // four FP32 vectors of nrhs * n_free
  if (rc) return rc;
  float* r32 = reinterpret_cast<float*>(pt->work);
  float* z32 = r32 + tot;
  float* t0 = z32 + tot;
  float* t1 = t0 + tot;
  launch_to_f32(r32, r, tot, st);
  if ((rc = pinv_apply_lp(pt, prec, nrhs, r32, z32, t0, t1, st))) return rc;
  launch_to_f64(z, z32, tot, st);
  return check_launch(0, "low-precision preconditioner");
}

int ga_patch_set_deterministic(ga_patch* pt, int on) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (pt->dim != 3) { set_error("the deterministic mode is for 3-D patches"); return GA_EINVAL; }
  pt->deterministic = on != 0;
  return GA_OK;
}

int ga_patch_set_layers(ga_patch* pt, int ze_mass, int ze_stiff) {
  if (!pt) { set_error("null patch"); return GA_EINVAL; }
  if (pt->dim != 3) { set_error("launch shapes are for 3-D patches"); return GA_EINVAL; }
  if (ze_mass < 0 || ze_mass > pt->n[2] || ze_stiff < 0 || ze_stiff > pt->n[2]) {
    set_error("layers per workgroup must be in 0..n_el[2]");
    return GA_EINVAL;
  }
  pt->ze_op[0] = ze_mass;
  pt->ze_op[1] = ze_stiff;
  return GA_OK;
}

int ga_mass_solve(ga_patch* pt, int nrhs, const double* b, double* x, double rtol, int maxit,
                  int prec, int* iters_out, double* relres_out, void* stream) {
  if (!pt || !b || !x) { set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1 || nrhs > 16) { set_error("nrhs must be in 1..16"); return GA_EINVAL; }
  if (!(rtol > 0.0) || maxit < 0) { set_error("rtol must be > 0 and maxit >= 0"); return GA_EINVAL; }
  if (prec != GA_FP64 && prec != GA_FP32 && prec != GA_BF16) { set_error("bad prec"); return GA_EINVAL; }
  if (prec != GA_FP64 && pt->dim != 3) { set_error("FP32 and BF16 solves need a 3-D patch"); return GA_EINVAL; }
  return solve_any(pt, nrhs, b, x, rtol, maxit, prec, false, iters_out, relres_out, S(stream));
}

int ga_lambda_max(ga_patch* pt, int iters, double* out, void* stream) {
  if (!pt || !out || iters < 1) { set_error("bad argument"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = pt->n_free;
  double *v = nullptr, *kv = nullptr, *u = nullptr, *mv = nullptr, *res = nullptr;
  int rc;
  if ((rc = dalloc((void**)&v, n * 8)) || (rc = dalloc((void**)&kv, n * 8)) ||
      (rc = dalloc((void**)&u, n * 8)) || (rc = dalloc((void**)&mv, n * 8)) ||
      (rc = dalloc((void**)&res, 64))) {
    hipFree(v); hipFree(kv); hipFree(u); hipFree(mv); hipFree(res);
    return rc;
  }
  std::vector<double> h(n);
  unsigned long long s = 0x9E3779B97F4A7C15ull;
  for (size_t i = 0; i < n; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    h[i] = (double)((s >> 11) & ((1ull << 52) - 1)) / (double)(1ull << 52) - 0.5;
  }
  hipMemcpy(v, h.data(), n * 8, hipMemcpyHostToDevice);
  double lam = 0.0;
  double hres[2];
  for (int it = 0; it < iters && rc == GA_OK; ++it) {
    launch_fill(kv, 0.0, n, st);
    if ((rc = op_apply(pt, 1, 1, 1.0, v, kv, st))) break;
    launch_fill(mv, 0.0, n, st);
    if ((rc = op_apply(pt, 0, 1, 1.0, v, mv, st))) break;
    launch_dot_partial(1, v, kv, n, pt->red, st);
    launch_sum_partials(1, pt->red, res, st);
    launch_dot_partial(1, v, mv, n, pt->red, st);
    launch_sum_partials(1, pt->red, res + 1, st);
    hipMemcpyAsync(hres, res, 16, hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    lam = hres[0] / hres[1];
    rc = solve_impl(pt, 1, kv, u, 1e-8, 500, true, nullptr, nullptr, st);
    if (rc == GA_ENOCONV) rc = GA_OK;
    if (rc) break;
    // normalise: v = u / sqrt(u.u)
    launch_dot_partial(1, u, u, n, pt->red, st);
    launch_sum_partials(1, pt->red, res, st);
    hipMemcpyAsync(hres, res, 8, hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    double nrm = std::sqrt(hres[0]);
    if (!(nrm > 0)) break;
    launch_axpby(v, 1.0 / nrm, u, 0.0, v, n, st);
  }
  hipFree(v); hipFree(kv); hipFree(u); hipFree(mv); hipFree(res);
  if (rc) return rc;
  *out = lam;
  return GA_OK;
}

int ga_integrator_create(ga_patch* pt, int k, double rho, double tau, double rtol, int maxit,
                         int prec, int guess_mode, ga_integrator** out) {
  if (!pt || !out) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  if (k < 1 || k > 4) { set_error("k must be in 1..4"); return GA_EINVAL; }
  if (!(rho >= 0.0 && rho < 1.0)) { set_error("rho must be in [0, 1)"); return GA_EINVAL; }
  if (!(tau > 0.0) || !(rtol > 0.0) || maxit < 1) { set_error("bad tau/rtol/maxit"); return GA_EINVAL; }
  if (guess_mode < GA_GUESS_ZERO || guess_mode > GA_GUESS_LEARNED) { set_error("bad guess mode"); return GA_EINVAL; }
  if (prec != GA_FP64 && prec != GA_FP32 && prec != GA_BF16) { set_error("bad prec"); return GA_EINVAL; }
  if (prec != GA_FP64 && pt->dim != 3) { set_error("mixed precision needs a 3-D patch"); return GA_EINVAL; }
  ga_integrator* it = new ga_integrator();
  it->prec = prec;
  it->patch = pt;
  it->k = k;
  it->rho = rho;
  it->tau = tau;
  it->rtol = rtol;
  it->maxit = maxit;
  it->guess = guess_mode;
  for (int j = 0; j < k; ++j) {
    if (j < k - 1) block_j_params(rho, it->alpha[j], it->beta[j], it->gamma[j]);
    else block_k_params(rho, it->alpha[j], it->beta[j], it->gamma[j]);
  }
  int rc;
  if ((rc = dalloc((void**)&it->Y, (size_t)k * pt->n_free * 8)) ||
      (rc = dalloc((void**)&it->Bv, (size_t)k * pt->n_free * 8)) ||
      (rc = dalloc((void**)&it->X, (size_t)k * pt->n_free * 8)) ||
      (rc = dalloc((void**)&it->H, (size_t)4 * k * pt->n_free * 8))) {
    ga_integrator_destroy(it);
    return rc;
  }
  *out = it;
  return GA_OK;
}

int ga_integrator_destroy(ga_integrator* it) {
  if (!it) return GA_OK;
  if (it->Y) hipFree(it->Y);
  if (it->Bv) hipFree(it->Bv);
  if (it->X) hipFree(it->X);
  if (it->H) hipFree(it->H);
  if (it->Z) hipFree(it->Z);
  delete it;
  return GA_OK;
}

int ga_integrator_set_net(ga_integrator* it, int stage, ga_gnet* net) {
  if (!it) { set_error("null integrator"); return GA_EINVAL; }
  if (stage < 0 || stage >= it->k) { set_error("stage out of range"); return GA_EINVAL; }
  if (net && it->patch->dim != 3) { set_error("the learned guess needs a 3-D patch"); return GA_EINVAL; }
  it->nets[stage] = net;
  return GA_OK;
}

int ga_integrator_history(const ga_integrator* it, int* nhist) {
  if (!it || !nhist) { set_error("null argument"); return GA_EINVAL; }
  *nhist = it->nhist;
  return GA_OK;
}

int ga_integrator_set_history(ga_integrator* it, int nhist, const double* const* hist,
                              void* stream) {
  if (!it || (nhist > 0 && !hist)) { set_error("null argument"); return GA_EINVAL; }
  if (nhist < 0 || nhist > 4) { set_error("nhist must be in 0..4"); return GA_EINVAL; }
  if (nhist > 0 && it->guess == GA_GUESS_ZERO) {
    set_error("a GA_GUESS_ZERO integrator keeps no history");
    return GA_EINVAL;
  }
  const int k = it->k;
  for (int i = 0; i < nhist * k; ++i)
    if (!hist[i]) { set_error("null history vector"); return GA_EINVAL; }
  const size_t n = it->patch->n_free;
  hipStream_t st = S(stream);
  // ring slots: the newest at head = nhist - 1, age a at head - a
  for (int a = 0; a < nhist; ++a)
    for (int j = 0; j < k; ++j)
      launch_copy(it->H + ((size_t)(nhist - 1 - a) * k + j) * n, hist[a * k + j], n, st);
  it->head = nhist > 0 ? nhist - 1 : -1;
  it->nhist = nhist;
  if (nhist > 0) launch_copy(it->X, it->H + (size_t)it->head * k * n, (size_t)k * n, st);
  it->have_prev = nhist > 0;
  return check_launch(0, "history restore");
}

int ga_stage_solution(ga_integrator* it, int stage, int age, double* out, void* stream) {
  if (!it || !out) { set_error("null argument"); return GA_EINVAL; }
  if (stage < 0 || stage >= it->k || age < 0 || age > 3) { set_error("stage or age out of range"); return GA_EINVAL; }
  const size_t n = it->patch->n_free;
  const double* src = nullptr;
  if (age < it->nhist) src = it->H + ((size_t)((it->head - age + 4) % 4) * it->k + stage) * n;
  else if (age == 0 && it->have_prev) src = it->X + (size_t)stage * n;
  if (!src) { set_error("no stage solution of that age yet"); return GA_EINVAL; }
  launch_copy(out, src, n, S(stream));
  return check_launch(0, "stage solution copy");
}

int ga_integrator_set_damping(ga_integrator* it, double cM, double cK) {
  if (!it) { set_error("null integrator"); return GA_EINVAL; }
  if (!(cM >= 0.0) || !(cK >= 0.0) || !std::isfinite(cM) || !std::isfinite(cK)) {
    set_error("damping coefficients must be finite and non-negative");
    return GA_EINVAL;
  }
  if (cM != 0.0 && !it->Z) {
    int rc = dalloc((void**)&it->Z, (size_t)it->k * it->patch->n_free * 8);
    if (rc) return rc;
  }
  it->cM = cM;
  it->cK = cK;
  return GA_OK;
}

int ga_stage_times(const ga_integrator* it, double t, double* out) {
  if (!it || !out) { set_error("null argument"); return GA_EINVAL; }
  for (int j = 0; j < it->k; ++j) out[j] = j < it->k - 1 ? t + it->tau : t;  // t_n + alpha_fj tau
  return GA_OK;
}

int ga_init_state_forced(ga_integrator* it, const double* U0, const double* V0,
                         const double* const* F0, double* const* state, void* stream) {
  if (!it || !U0 || !V0 || !state) { set_error("null argument"); return GA_EINVAL; }
  const int N = 3 * it->k - 3;
  for (int s = 0; s < 3 * it->k; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  if (F0)
    for (int a = 0; a <= N; ++a)
      if (!F0[a]) { set_error("null forcing vector"); return GA_EINVAL; }
  ga_patch* pt = it->patch;
  hipStream_t st = S(stream);
  const size_t n = pt->n_free;
  launch_copy(state[0], U0, n, st);
  launch_copy(state[1], V0, n, st);
  // L^a = M^{-1}(F^{(a)}(0) - C L^{a-1} - K L^{a-2}), C = cM M + cK K
  for (int a = 0; a <= N; ++a) {
    double* rhs = it->Bv;
    double* karg = it->Y;
    if (it->cK != 0.0) launch_axpby(karg, 1.0, state[a], it->cK, state[a + 1], n, st);
    else launch_copy(karg, state[a], n, st);
    if (F0) launch_copy(rhs, F0[a], n, st);
    else launch_fill(rhs, 0.0, n, st);
    int rc = op_apply(pt, 1, 1, -1.0, karg, rhs, st);
    if (rc) return rc;
    if (it->cM != 0.0 && (rc = op_apply(pt, 0, 1, -it->cM, state[a + 1], rhs, st))) return rc;
    rc = solve_any(pt, 1, rhs, state[a + 2], it->rtol, it->maxit, it->prec, true, nullptr,
                   nullptr, st);
    if (rc) return rc;
  }
  it->have_prev = false;
  it->head = -1;
  it->nhist = 0;
  return GA_OK;
}

int ga_init_state(ga_integrator* it, const double* U0, const double* V0, double* const* state,
                  void* stream) {
  return ga_init_state_forced(it, U0, V0, nullptr, state, stream);
}

}  // extern "C"

namespace {

// one step: predictors, stage right-hand sides b_j = F_j - C Z_j - K Y_j (eq. ho1;
// F optional, C = cM M + cK K), the k solves and the update
int step_once(ga_integrator* it, const StatePtrs& sp, const Coefs& cf, const double* const* F,
              int* iters, hipStream_t st) {
  ga_patch* pt = it->patch;
  const int k = it->k;
  const size_t n = pt->n_free;
  const bool damped = it->cM != 0.0 || it->cK != 0.0;
  if (damped) launch_predict_cz(k, it->tau, it->cK, sp, it->Y, it->cM != 0.0 ? it->Z : nullptr, n, st);
  else launch_predict(k, it->tau, sp, it->Y, n, st);
  if (F)
    for (int j = 0; j < k; ++j) launch_copy(it->Bv + (size_t)j * n, F[j], n, st);
  else
    launch_fill(it->Bv, 0.0, (size_t)k * n, st);
  int rc = op_apply(pt, 1, k, -1.0, it->Y, it->Bv, st);
  if (rc) return rc;
  if (it->cM != 0.0 && (rc = op_apply(pt, 0, k, -it->cM, it->Z, it->Bv, st))) return rc;
  // initial guess from the history of stage solutions (newest first)
  bool zero = true;
  if (it->guess != GA_GUESS_ZERO && it->nhist > 0) {
    const int nh = it->guess == GA_GUESS_PREV ? 1 : it->nhist;
    const double* hp[16] = {nullptr};
    for (int h = 0; h < nh; ++h)
      for (int j = 0; j < k; ++j)
        hp[h * 4 + j] = it->H + ((size_t)((it->head - h + 4) % 4) * k + j) * n;
    // stages with a net get their guess (which contains the extrapolation) from the
    // net's kernels alone; the others take the extrapolation
    bool all_nets = it->guess == GA_GUESS_LEARNED && it->nhist == 4;
    for (int j = 0; j < k && all_nets; ++j) all_nets = it->nets[j] != nullptr;
    if (!all_nets) launch_extrap(k, nh, hp, it->X, n, st);
    if (it->guess == GA_GUESS_LEARNED && it->nhist == 4) {
      for (int j = 0; j < k; ++j) {
        if (!it->nets[j]) continue;
        const double* hj[4] = {hp[j], hp[4 + j], hp[8 + j], hp[12 + j]};
        ProfScope prof(3, st);
        rc = gnet_guess(it->nets[j], pt, hj, it->X + (size_t)j * n, st);
        if (rc) return rc;
      }
    }
    zero = false;
  }
  rc = solve_any(pt, k, it->Bv, it->X, it->rtol, it->maxit, it->prec, zero, iters, nullptr, st);
  if (rc) return rc;
  if (it->guess != GA_GUESS_ZERO) {  // push the solutions into the history ring
    it->head = (it->head + 1) % 4;
    launch_copy(it->H + (size_t)it->head * k * n, it->X, (size_t)k * n, st);
    it->nhist = std::min(it->nhist + 1, 4);
  }
  launch_update(k, it->tau, cf, sp, it->X, n, st);
  if (check_launch(0, "update")) return GA_EDEVICE;
  it->have_prev = true;
  return GA_OK;
}

// |U|^2 and |V|^2 of a state into scal slots dst, dst + 1 (enqueued, no host read)
constexpr int GROWTH_SLOT = NSCAL * 63;
void launch_state_norms(ga_patch* pt, const double* u, const double* v, double* dst,
                        hipStream_t st) {
  double* part = pt->red;
  launch_dot_partial(1, u, u, pt->n_free, part, st);
  launch_dot_partial(1, v, v, pt->n_free, part + RED_BLOCKS, st);
  launch_sum_partials(2, part, dst, st);
}

// after nsteps unforced steps: non-finite U or V, or N = |U| + tau |V| grown by more
// than 10 * 1.05^nsteps since the norms taken before the steps (slots +2, +3), is
// GA_EUNSTABLE.  A stable step keeps the discrete energy bounded; N can still grow
// from a small start (U0 = 0: N_n ~ (n + 1) N_0 while n tau omega << 1), which the
// bound admits for every n, while an unstable mode grows geometrically.
int check_growth(ga_integrator* it, const double* u, const double* v, int nsteps,
                 hipStream_t st) {
  ga_patch* pt = it->patch;
  double* slot = pt->scal + GROWTH_SLOT;
  launch_state_norms(pt, u, v, slot, st);
  double h[4];
  GA_TRY_HIP(hipMemcpyAsync(h, slot, sizeof(h), hipMemcpyDeviceToHost, st));
  GA_TRY_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) {
    set_error("displacement or velocity became non-finite");
    return GA_EUNSTABLE;
  }
  const double n1 = std::sqrt(h[0]) + it->tau * std::sqrt(h[1]);
  const double n0 = std::sqrt(h[2]) + it->tau * std::sqrt(h[3]);
  if (n0 > 0.0 && std::log(n1 / n0) > std::log(10.0) + nsteps * std::log(1.05)) {
    char msg[160];
    snprintf(msg, sizeof(msg),
             "|U| + tau |V| grew by %.3g over %d steps: beyond the growth of a stable step",
             n1 / n0, nsteps);
    set_error(msg);
    return GA_EUNSTABLE;
  }
  return GA_OK;
}

int check_finite(ga_patch* pt, const double* u, hipStream_t st) {
  double* part = pt->red;
  launch_dot_partial(1, u, u, pt->n_free, part, st);
  launch_sum_partials(1, part, pt->scal + NSCAL * 63, st);
  double nrm2 = 0.0;
  GA_TRY_HIP(hipMemcpyAsync(&nrm2, pt->scal + NSCAL * 63, 8, hipMemcpyDeviceToHost, st));
  GA_TRY_HIP(hipStreamSynchronize(st));
  if (!std::isfinite(nrm2)) { set_error("displacement became non-finite"); return GA_EUNSTABLE; }
  return GA_OK;
}

int step_setup(ga_integrator* it, double* const* state, StatePtrs& sp, Coefs& cf) {
  const int k = it->k, ns = 3 * k;
  for (int s = 0; s < ns; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  for (int s = 0; s < 12; ++s) sp.L[s] = s < ns ? state[s] : nullptr;
  for (int j = 0; j < 4; ++j) {
    cf.alpha[j] = j < k ? it->alpha[j] : 1.0;
    cf.beta[j] = j < k ? it->beta[j] : 0.0;
    cf.gamma[j] = j < k ? it->gamma[j] : 0.0;
  }
  return GA_OK;
}

}  // namespace

extern "C" {

int ga_step(ga_integrator* it, double* const* state, int nsteps, int* iters_out, void* stream) {
  if (!it || !state || nsteps < 0) { set_error("bad argument"); return GA_EINVAL; }
  StatePtrs sp;
  Coefs cf;
  int rc = step_setup(it, state, sp, cf);
  if (rc) return rc;
  hipStream_t st = S(stream);
  launch_state_norms(it->patch, state[0], state[1], it->patch->scal + GROWTH_SLOT + 2, st);
  int iters[16];
  for (int step = 0; step < nsteps; ++step) {
    if ((rc = step_once(it, sp, cf, nullptr, iters, st))) return rc;
    if (iters_out)
      for (int j = 0; j < it->k; ++j) iters_out[(size_t)step * it->k + j] = iters[j];
  }
  return check_growth(it, state[0], state[1], nsteps, st);
}

int ga_step_forced(ga_integrator* it, double* const* state, const double* const* forcing,
                   int* iters_out, void* stream) {
  if (!it || !state || !forcing) { set_error("null argument"); return GA_EINVAL; }
  for (int j = 0; j < it->k; ++j)
    if (!forcing[j]) { set_error("null forcing vector"); return GA_EINVAL; }
  StatePtrs sp;
  Coefs cf;
  int rc = step_setup(it, state, sp, cf);
  if (rc) return rc;
  hipStream_t st = S(stream);
  if ((rc = step_once(it, sp, cf, forcing, iters_out, st))) return rc;
  return check_finite(it->patch, state[0], st);
}

}  // extern "C"
