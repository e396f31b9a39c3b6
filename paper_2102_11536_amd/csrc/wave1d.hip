// Batched 1-D wave problems for the dispersion study (Sec. 6.2): R independent
// systems M U_r'' + omega_r^2 K U_r = 0 on (0, 1) with homogeneous Dirichlet
// data, splines of degree p on n uniform elements (identity map), all stepped
// by the order-2k scheme with one tau.  Each system is one wavenumber of the
// study; batching them turns R tiny launch-bound runs into one run.
//
// Layout: a batched vector holds system r at entries r*m .. r*m+m-1 (m = n+p-2
// free coefficients); the k stage vectors are R*m entries apart, so the k*R
// stage systems are the rows of one [k*R][m] matrix.
//
// One step is four launches and no host synchronisation:
//   predict_k      Taylor predictors Y_j (shared with the 3-D path);
//   band_mv_k      b_j = -omega_r^2 K Y_j with the banded K (bandwidth p);
//   gemm_f64_k     X = B M^{-1}: on the identity map the Kronecker
//                  preconditioner of Sec. 5.4 is M itself (D = diag M /
//                  diag M-hat = 1), so PCG stops at its first iterate, which
//                  is M^{-1} b; it is applied as one FP64 GEMM with the dense
//                  inverse over all k*R rows;
//   update_k       the 3k-vector update (shared with the 3-D path).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "ga_internal.h"
#include "kernels.h"

using namespace ga;

struct ga_wave1d {
  int n = 0, p = 0, m = 0, R = 0, k = 1;
  double rho_b = 0.5, rho_s = 0.5, tau = 0.0;
  Coefs cf{};
  double *Kb = nullptr, *Mb = nullptr;   // [m][2p+1] bands of K and M
  double* Minv = nullptr;                // [m][m] dense inverse of M
  double* w2 = nullptr;                  // [R] omega_r^2
  double *Y = nullptr, *Bv = nullptr, *X = nullptr;   // [k][R][m]
  std::vector<double> w2_host;
};

namespace {

constexpr int VB = 256;

// y[s][i] = alpha * c[s % R] * sum_d A[i][d] x[s][i - p + d]   (s < ns systems)
__global__ void __launch_bounds__(VB)
band_mv_k(const double* __restrict__ A, int m, int p, int R, const double* __restrict__ x,
          double* __restrict__ y, const double* __restrict__ c, double alpha, long long total) {
  for (long long t = (long long)blockIdx.x * VB + threadIdx.x; t < total;
       t += (long long)gridDim.x * VB) {
    const long long s = t / m;
    const int i = (int)(t - s * m);
    const double* xs = x + s * m;
    const double* a = A + (size_t)i * (2 * p + 1);
    double acc = 0.0;
    for (int d = 0; d <= 2 * p; ++d) {
      const int j = i - p + d;
      if (j >= 0 && j < m) acc += a[d] * xs[j];
    }
    y[t] = alpha * (c ? c[s % R] : 1.0) * acc;
  }
}

unsigned blocks_for(long long n) {
  long long b = (n + VB - 1) / VB;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

void band_mv(const ga_wave1d* w, const double* A, int ns, const double* x, double* y,
             const double* c, double alpha, hipStream_t st) {
  const long long total = (long long)ns * w->m;
  hipLaunchKernelGGL(band_mv_k, dim3(blocks_for(total)), dim3(VB), 0, st, A, w->m, w->p, w->R, x, y,
                     c, alpha, total);
}

// X[s] = M^{-1} B[s] for ns rows (M symmetric: X = B M^{-1} row by row)
void mass_solve(const ga_wave1d* w, int ns, const double* B, double* X, hipStream_t st) {
  launch_gemm(ns, w->m, w->m, B, w->m, 0, w->Minv, w->m, 0, X, w->m, 0, 1, st);
}

// banded storage [m][2p+1] (column j = i - p + d) of a symmetric matrix given by
// its Gauss-point products on the free coefficients 1 .. m
std::vector<double> band_of(const Axis1D& ax, bool stiff) {
  const int p = ax.p, P1 = p + 1, W = 2 * p + 1, m = ax.mf;
  std::vector<double> A((size_t)m * W, 0.0);
  for (int e = 0; e < ax.n; ++e)
    for (int q = 0; q < ax.q; ++q) {
      const double* f = stiff ? &ax.D[((size_t)e * ax.q + q) * P1] : &ax.B[((size_t)e * ax.q + q) * P1];
      const double wq = ax.w[(size_t)e * ax.q + q];
      for (int r = 0; r < P1; ++r)
        for (int c = 0; c < P1; ++c) {
          const int i = e + r - ax.lo, j = e + c - ax.lo;
          if (i < 0 || j < 0 || i >= m || j >= m) continue;
          A[(size_t)i * W + (j - i + p)] += wq * f[r] * f[c];
        }
    }
  return A;
}

void free_wave(ga_wave1d* w) {
  for (void* p : {(void*)w->Kb, (void*)w->Mb, (void*)w->Minv, (void*)w->w2, (void*)w->Y,
                  (void*)w->Bv, (void*)w->X})
    if (p) hipFree(p);
  delete w;
}

int upload(double** dst, const std::vector<double>& v) {
  int rc = dalloc((void**)dst, v.size() * sizeof(double));
  if (rc) return rc;
  GA_TRY_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  return GA_OK;
}

}  // namespace

extern "C" {

double ga_stability_limit2(double rho_b, double rho_s) {
  double a, b, g;
  block_k_params2(rho_b, rho_s, a, b, g);
  return (4.0 * a - 2.0) / (2.0 * b - g);
}

int ga_wave1d_create(int n_el, int p, int nsys, const double* omega2_host, int k, double rho_b,
                     double rho_s, double tau, ga_wave1d** out) {
  if (!out || !omega2_host) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  if (n_el < 1 || p < 1 || p > 4 || n_el + p - 2 < 1) { set_error("need n_el >= 1 and p in 1..4"); return GA_EINVAL; }
  if (nsys < 1 || k < 1 || k > 4) { set_error("need nsys >= 1 and k in 1..4"); return GA_EINVAL; }
  if (!(rho_b >= 0.0 && rho_b < 1.0) || !(rho_s >= 0.0 && rho_s <= rho_b) || !(tau > 0.0)) {
    set_error("need 0 <= rho_s <= rho_b < 1 and tau > 0");
    return GA_EINVAL;
  }
  for (int r = 0; r < nsys; ++r)
    if (!(omega2_host[r] > 0.0) || !std::isfinite(omega2_host[r])) {
      set_error("omega^2 must be positive and finite");
      return GA_EINVAL;
    }
  ga_wave1d* w = new ga_wave1d();
  w->n = n_el;
  w->p = p;
  w->m = n_el + p - 2;
  w->R = nsys;
  w->k = k;
  w->rho_b = rho_b;
  w->rho_s = rho_s;
  w->tau = tau;
  w->w2_host.assign(omega2_host, omega2_host + nsys);
  for (int j = 0; j < 4; ++j) {
    double a = 1.0, b = 0.0, g = 0.0;
    if (j < k - 1) block_j_params2(rho_b, rho_s, a, b, g);
    else if (j == k - 1) block_k_params2(rho_b, rho_s, a, b, g);
    w->cf.alpha[j] = a;
    w->cf.beta[j] = b;
    w->cf.gamma[j] = g;
  }
  const Axis1D ax = build_axis(n_el, p, 1, w->m);
  const size_t kn = (size_t)k * nsys * w->m;
  int rc;
  if ((rc = upload(&w->Kb, band_of(ax, true))) || (rc = upload(&w->Mb, band_of(ax, false))) ||
      (rc = upload(&w->Minv, ax.Minv)) || (rc = upload(&w->w2, w->w2_host)) ||
      (rc = dalloc((void**)&w->Y, kn * 8)) || (rc = dalloc((void**)&w->Bv, kn * 8)) ||
      (rc = dalloc((void**)&w->X, kn * 8))) {
    free_wave(w);
    return rc;
  }
  *out = w;
  return GA_OK;
}

int ga_wave1d_destroy(ga_wave1d* w) {
  if (!w) return GA_OK;
  hipDeviceSynchronize();
  free_wave(w);
  return GA_OK;
}

int ga_wave1d_info(const ga_wave1d* w, int* n_free) {
  if (!w) { set_error("null handle"); return GA_EINVAL; }
  if (n_free) *n_free = w->m;
  return GA_OK;
}

int ga_wave1d_load_sine(ga_wave1d* w, const double* wavenumbers, double* f, void* stream) {
  if (!w || !wavenumbers || !f) { set_error("null argument"); return GA_EINVAL; }
  // f[r][i] = int_0^1 b_i sin(j_r pi x) dx with 2p + 8 Gauss points per element
  const int nq = 2 * w->p + 8, P1 = w->p + 1, m = w->m;
  std::vector<double> t, wt, host((size_t)w->R * m, 0.0);
  gauss_legendre01(nq, t, wt);
  double val[8], der[8];
  for (int e = 0; e < w->n; ++e)
    for (int q = 0; q < nq; ++q) {
      const double x = (e + t[q]) / w->n, wq = wt[q] / w->n;
      basis_on_element(w->n, w->p, e, x, val, der);
      for (int r = 0; r < w->R; ++r) {
        const double s = wq * std::sin(wavenumbers[r] * M_PI * x);
        for (int c = 0; c < P1; ++c) {
          const int i = e + c - 1;
          if (i >= 0 && i < m) host[(size_t)r * m + i] += s * val[c];
        }
      }
    }
  GA_TRY_HIP(hipMemcpyAsync(f, host.data(), host.size() * 8, hipMemcpyHostToDevice, S(stream)));
  GA_TRY_HIP(hipStreamSynchronize(S(stream)));
  return GA_OK;
}

int ga_wave1d_apply(ga_wave1d* w, char which, const double* x, double* y, void* stream) {
  if (!w || !x || !y) { set_error("null argument"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  if (which == 'M') band_mv(w, w->Mb, w->R, x, y, nullptr, 1.0, st);
  else if (which == 'K') band_mv(w, w->Kb, w->R, x, y, nullptr, 1.0, st);
  else if (which == 'S') mass_solve(w, w->R, x, y, st);
  else { set_error("which must be 'M', 'K' or 'S'"); return GA_EINVAL; }
  return check_launch(0, "1-D apply");
}

int ga_wave1d_init_state(ga_wave1d* w, const double* U0, const double* V0, double* const* state,
                         void* stream) {
  if (!w || !U0 || !V0 || !state) { set_error("null argument"); return GA_EINVAL; }
  for (int s = 0; s < 3 * w->k; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = (size_t)w->R * w->m;
  launch_copy(state[0], U0, n, st);
  launch_copy(state[1], V0, n, st);
  // L^a = M^{-1} (-omega^2 K L^{a-2}), a = 0 .. 3k-3
  for (int a = 0; a <= 3 * w->k - 3; ++a) {
    band_mv(w, w->Kb, w->R, state[a], w->Bv, w->w2, -1.0, st);
    mass_solve(w, w->R, w->Bv, state[a + 2], st);
  }
  return check_launch(0, "1-D initial state");
}

int ga_wave1d_step(ga_wave1d* w, double* const* state, int nsteps, void* stream) {
  if (!w || !state || nsteps < 0) { set_error("bad argument"); return GA_EINVAL; }
  const int k = w->k;
  for (int s = 0; s < 3 * k; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = (size_t)w->R * w->m;
  StatePtrs sp;
  for (int s = 0; s < 12; ++s) sp.L[s] = s < 3 * k ? state[s] : nullptr;
  for (int i = 0; i < nsteps; ++i) {
    launch_predict(k, w->tau, sp, w->Y, n, st);
    band_mv(w, w->Kb, k * w->R, w->Y, w->Bv, w->w2, -1.0, st);
    mass_solve(w, k * w->R, w->Bv, w->X, st);
    launch_update(k, w->tau, w->cf, sp, w->X, n, st);
  }
  return check_launch(0, "1-D step");
}

}  // extern "C"
