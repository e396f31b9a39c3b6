// Internal declarations of the ga library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>
#include <vector>

#include "../../include/ga.h"

namespace ga {

// Univariate data of one tensor axis.
struct Axis1D {
  int n = 0, p = 0, q = 0, m = 0, mf = 0, lo = 1;
  std::vector<double> B, D;   // [n][q][p+1]: values / derivatives of basis e+r at Gauss point j of element e
  std::vector<double> w;      // [n][q]: Gauss weights (element length included)
  std::vector<double> dhat;   // [mf]: diagonal of the univariate parametric mass (free part)
  std::vector<double> Minv;   // [mf][mf]: its dense inverse, row-major
  // its banded Cholesky factor L (bandwidth p), [mf + p][p + 1]: entry d = 0 holds
  // 1 / L(i,i), entry d >= 1 holds L(i, i-d); the p trailing rows are zero
  std::vector<double> chol;
};

// free coefficients lo .. lo+mf_free-1 of the n+p along the axis (lo = 1, mf_free =
// n+p-2 when both ends carry homogeneous Dirichlet data)
Axis1D build_axis(int n, int p, int lo, int mf_free);
void gauss_legendre01(int nq, std::vector<double>& t, std::vector<double>& w);
void basis_on_element(int n, int p, int e, double x, double* val, double* der);

// Element tile of the sum-factorised operator kernels: TE elements per
// direction, quadrature factors stored tile by tile.
// 3-D: elements per xy-column edge of the stiffness and the mass kernels
// (at most 1024 threads = (TE*(p+1))^2 per workgroup); measured on MI355X:
// 4 x 4 columns for p <= 3, 3 x 3 for p = 4 (225 threads instead of 400)
#ifndef GA_TES2
#define GA_TES2 4
#endif
#ifndef GA_TES4
#define GA_TES4 3
#endif
constexpr int te3_stiff(int p) { return p == 2 ? GA_TES2 : (p == 4 ? GA_TES4 : 4); }
#ifndef GA_TE3_MASS
#define GA_TE3_MASS 4
#endif
#ifndef GA_TEM2
#define GA_TEM2 GA_TE3_MASS
#endif
#ifndef GA_TEM4
#define GA_TEM4 3
#endif
constexpr int te3_mass_raw(int p) { return p == 2 ? GA_TEM2 : (p == 4 ? GA_TEM4 : GA_TE3_MASS); }
constexpr int te3_mass(int p) { return (p + 1) * te3_mass_raw(p) > 32 ? 32 / (p + 1) : te3_mass_raw(p); }
constexpr int TE2 = 8;   // 2-D tile: 8 x 8 elements

void set_error(const std::string& msg);

#define GA_TRY_HIP(call)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) {                                                                \
      ga::set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_));  \
      return GA_EDEVICE;                                                                   \
    }                                                                                      \
  } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int dalloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc failed (" + std::to_string(bytes) + " bytes)");
    return GA_ENOMEM;
  }
  return GA_OK;
}

inline int check_launch(int rc, const char* what) {
  hipError_t e = hipGetLastError();
  if (rc != 0 || e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + what + " (" + hipGetErrorString(e) + ")");
    return GA_EDEVICE;
  }
  return GA_OK;
}

// parameters (alpha, beta, gamma) of the blocks j < k and of block k of the
// order-2k scheme with rho_b = rho_s = rho
void block_j_params(double rho, double& a, double& b, double& g);
void block_k_params(double rho, double& a, double& b, double& g);
// the two-parameter family rho_s <= rho_b (type-j formulas at (-rho_b, -rho_s),
// type-k at (rho_b, rho_s))
void block_j_params2(double rho_b, double rho_s, double& a, double& b, double& g);
void block_k_params2(double rho_b, double rho_s, double& a, double& b, double& g);

// FP32 copies of a 3-D patch's factors, 1-D inverses, band factors and scaling
// for the mixed-precision solves (built once, kept with the patch)
int mixed_setup(ga_patch* pt, hipStream_t st);

// FP64 P^{-1} with caller-provided scratch vectors t0, t1 (nr * n_free each); no
// allocation
int pinv_apply_scratch(ga_patch* pt, int nr, const double* r, double* z, double* t0, double* t1,
                       hipStream_t st);

// whole-grid learned guess of one stage from its four newest solutions h[0..3]
int gnet_guess(ga_gnet* net, ga_patch* pt, const double* const* h, double* X, hipStream_t st);

}  // namespace ga

struct ga_patch {
  int dim = 0, p = 0;
  int n[3] = {1, 1, 1}, m[3] = {1, 1, 1}, mf[3] = {1, 1, 1};
  int lo[3] = {1, 1, 1};          // first free coefficient per axis (0: that face is free)
  int nt[3] = {1, 1, 1};          // element tiles per direction (2-D kernels)
  int ntk[2] = {1, 1}, ntm[2] = {1, 1};  // 3-D xy columns: stiffness and mass layouts
  int ze = 0;                     // element layers per workgroup along z (0: automatic)
  int ze_op[2] = {0, 0};          // tuned layers for the mass / stiffness kernels (0: automatic)
  int pinv_mode = GA_PINV_AUTO;   // preconditioner algorithm (ga_patch_set_pinv)
  int cg_ctrl = GA_CG_DEVICE;     // PCG control (ga_patch_set_cg)
  bool deterministic = false;     // colour-ordered operator launches (ga_patch_set_deterministic)
  int hint_nr = 0;                // iterations per right-hand side of the last FP64 solve
  int hint[16] = {0};             //   of hint_nr right-hand sides (speculative schedule)
  long long n_spec = 0, n_checks = 0;   // iterations enqueued ahead, host convergence reads
  int mx_hint[2] = {0, 0};        // inner iterations per pass of the last FP32 / BF16 mixed solve
  long long n_free = 0, n_quad = 0, n_tiles = 0, qp_per_tile = 0;
  ga::Axis1D ax[3];
  // device data
  double* tabB[3] = {nullptr, nullptr, nullptr};   // [n_pad][q][p+1]
  double* tabD[3] = {nullptr, nullptr, nullptr};
  double* tabB2[3] = {nullptr, nullptr, nullptr};  // squared values (diag(M))
  double* W = nullptr;        // w |det J|            (3-D: mass-kernel column layout)
  double* G = nullptr;        // w |det J| J^-1 J^-T  (3-D: stiffness-kernel column layout)
  size_t nW = 0, nG = 0;      // entries
  float* W32 = nullptr;       // FP32 copy of W (mixed-precision inner solves)
  float* G32 = nullptr;       // FP32 copy of G (FP32 stiffness applies)
  unsigned short* W16 = nullptr;  // BF16 copies of W and G (bit patterns, round to nearest even)
  unsigned short* G16 = nullptr;
  float* Minv32[3] = {nullptr, nullptr, nullptr};  // FP32 copies of the 1-D inverses
  float* s32 = nullptr;       // FP32 copy of the scaling
  double* cb[3] = {nullptr, nullptr, nullptr};    // banded Cholesky factors (Axis1D::chol)
  float* cb32[3] = {nullptr, nullptr, nullptr};
  double* diagM = nullptr;    // [n_free]
  double* s = nullptr;        // [n_free] (Dhat/D)^(1/2)
  double* Minv[3] = {nullptr, nullptr, nullptr};   // [mf][mf]
  void* apk[3][3] = {};       // [prec][axis]: the inverses packed for the matrix cores
  // work buffers for solves (grown on demand)
  double* work = nullptr;
  size_t work_bytes = 0;
  double* red = nullptr;      // reduction partials
  double* scal = nullptr;     // device scalars
  int* flags = nullptr;       // device flags
  double* cgf_part = nullptr;  // fused-reduction partials of the single-reduction PCG
  unsigned* cgf_cnt = nullptr; // and its last-workgroup counters
  double* host_scal = nullptr;  // pinned host mirror of scalars
  // solve statistics
  long long n_solves = 0, n_guessed = 0, n_fallbacks = 0;
  double guess_rel_sum = 0.0;   // sum over guessed solves of |r0|_P / |b|_P
};

struct ga_integrator {
  ga_patch* patch = nullptr;
  int k = 1;
  double rho = 0.5, tau = 0.0, rtol = 1e-10;
  int maxit = 200, guess = GA_GUESS_ZERO, prec = GA_FP64;
  double alpha[8], beta[8], gamma[8];
  double* Y = nullptr;        // [k][n_free] stage arguments Y_j
  double* Bv = nullptr;       // [k][n_free] stage right-hand sides -K Y_j
  double* X = nullptr;        // [k][n_free] stage solutions
  double* H = nullptr;        // [4][k][n_free] ring of past stage solutions
  double* Z = nullptr;        // [k][n_free] damping arguments (Rayleigh mass part)
  double cM = 0.0, cK = 0.0;  // Rayleigh damping C = cM M + cK K
  int head = -1, nhist = 0;   // newest ring slot, number of valid slots
  bool have_prev = false;
  ga_gnet* nets[4] = {nullptr, nullptr, nullptr, nullptr};  // learned guess per stage (not owned)
};

struct ga_gnet {
  float* params = nullptr;    // FP32 master weights, tap-major layout
  float* m = nullptr;         // Adam moments
  float* v = nullptr;
  long long adam_t = 0;
  void* wpk = nullptr;        // BF16 inference weights of the three layers, packed
  bool packed = false;
  float* tw = nullptr;        // training activations and gradients
  size_t tw_bytes = 0;
  int* org = nullptr;         // crop origins [nb][3]
  int org_cap = 0;
  double* scal = nullptr;     // [0..3]: sums of squares of the history differences D_0..D_3
  double* part = nullptr;     // reduction partials
  void* iw = nullptr;         // inference activations (BF16, channels-last)
  int train_prec = GA_BF16;   // GA_BF16: layer 2 of training on MFMA; GA_FP32: all FP32
  size_t iw_bytes = 0;
};
