// Launchers shared between the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>

#include "ga_internal.h"

namespace ga {

constexpr int RED_BLOCKS = 256;   // partial sums per reduction
constexpr int NSCAL = 12;         // device scalars per right-hand side
enum { S_RZ = 0, S_PQ = 1, S_ALPHA = 2, S_BETA = 3, S_BN2 = 4, S_ACTIVE = 5, S_ITERS = 6, S_TOL2 = 7,
       S_FALLBACK = 8, S_RZ0 = 9 };
// single-reduction PCG (Chronopoulos-Gear): alpha and gamma of the previous update,
// in two slots each, alternated by the parity of the iteration (the update kernel
// reads one and its first workgroup writes the other)
enum { S_ALPHA0 = 2, S_ALPHA1 = 3, S_GPREV0 = 1, S_GPREV1 = 11 };

// Reductions fused into a producing kernel: every workgroup writes its partial sum
// part[rhs * pstride + wg]; the last workgroup to finish (counted in cnt[slot]) sums
// them in workgroup order (the same order every run) and updates the scalars.
struct CgFuse {
  double* part;
  unsigned* cnt;
  double* scal;       // CG scalars of right-hand side 0 of the launch
  long long pstride;  // partial slots per right-hand side
};
constexpr long long CGF_PSTRIDE = 65536;  // partial slots per right-hand side
constexpr int CGF_MAXRHS = 16;

// after z = P^{-1} r: gamma = r^T z and the stopping test of the solve
__device__ inline void cgcg_gamma(double* s, double gamma) {
  if (s[S_ACTIVE] == 0.0) return;
  s[S_RZ] = gamma;
  if (!(gamma > s[S_TOL2] * s[S_BN2])) s[S_ACTIVE] = 0.0;
}
// the last-workgroup reduction of a fused dot: called by every thread of the
// workgroup after its partials part[r * pstride + wg] (r < nr) are written by thread
// 0; `done` (an LDS int) and `sh` (LDS, >= blockDim.x / 64 doubles) are scratch.
// Returns in the last workgroup, with the totals applied by `apply(r, total)` on
// thread 0.
template <class F>
__device__ inline void cgf_finish(const CgFuse& f, unsigned slot, unsigned nwg, int nr, int* done,
                                  double* sh, F apply) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(&f.cnt[slot], 1u);
    *done = prev == nwg - 1;
  }
  __syncthreads();
  if (!*done) return;
  __threadfence();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int r = 0; r < nr; ++r) {
    double v = 0.0;
    for (unsigned i = threadIdx.x; i < nwg; i += blockDim.x)
      v += __builtin_nontemporal_load(&f.part[(long long)r * f.pstride + i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < nw; ++i) t += sh[i];
      apply(r, t);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) f.cnt[slot] = 0u;   // ready for the next launch
}

struct StatePtrs { double* L[12]; };
struct HistPtrs { const double* H[16]; };  // [h * 4 + j]: history slot h (newest first), stage j
struct Coefs { double alpha[4], beta[4], gamma[4]; };

// element/tile geometry of one 3-D patch as the operator kernels see it
struct Geo3 {
  int n[3], m[3], mf[3], nt[2], lo[3];
};

// one patch of a multi-patch operator launch (all patches of one degree)
struct OpGroupEntry {
  const void* fac;            // W (mass, FP64 or FP32) or G (stiffness) of the patch
  const double* tB[3];
  const double* tD[3];
  Geo3 g;
  int ze;                     // element layers per tile along z
  long long off;              // offset of the patch's segment in the batched vectors
  int tile0, ntiles;          // the patch's entries in the tile queue
  int sys;                    // the patch's index in the batch (its systems j * R + sys)
};

// device-side control of a batched launch: the right-hand side j (j0 + j within the
// launch) of the patch with index sys is system (j0 + j) * R + sys, whose CG scalars
// are scal + system * NSCAL; work of systems that have all converged is skipped
struct BatchGate {
  const double* scal;   // null: no gating
  int R, j0;
};
__device__ inline bool batch_active(const BatchGate& g, int sys, int j) {
  return !g.scal || g.scal[(size_t)((g.j0 + j) * g.R + sys) * NSCAL + S_ACTIVE] != 0.0;
}

int launch_op3d(int mode, int nr, const ga_patch* pt, const double* x, double* y, double alpha,
                hipStream_t st,
                const double* gate = nullptr);
long long op3d_tiles(int mode, const ga_patch* pt, int ze);
// right-hand sides per operator launch: 3, except the p = 4 stiffness, whose
// three-right-hand-side kernel spills registers (measured at 128^3: NR = 3
// 16.9 ms, NR = 2 + NR = 1 8.3 ms)
inline int op3d_max_nr(int p, int mode) { return (mode == 1 && p == 4) ? 2 : 3; }
int op3d_default_ze(int mode, const ga_patch* pt, bool f32 = false);
OpGroupEntry op3d_group_entry(int mode, const ga_patch* pt, int ze, long long off, int tile0,
                              bool f32);
// y += alpha * Op x over every patch in ents (one degree p), nr right-hand sides
// `stride` entries apart, the tile queue split over at most nwg workgroups
template <typename S>
int launch_op3d_group(int p, int mode, int nr, const OpGroupEntry* ents, int nent, const S* x,
                      S* y, long long stride, S alpha, int total, int nwg, hipStream_t st,
                      BatchGate gate = BatchGate{nullptr, 0, 0});
int launch_mass3d_f32(int nr, const ga_patch* pt, const float* x, float* y, float alpha,
                      hipStream_t st);
// FP32-vector operator apply (mode 0 mass, 1 stiffness) with FP32 (prec GA_FP32:
// W32, G32) or BF16 (GA_BF16: W16, G16) factors; -1 if those factors are not built
int launch_op3d_lowp(int mode, int nr, const ga_patch* pt, const float* x, float* y, float alpha,
                     int prec, hipStream_t st, const double* gate = nullptr);
int launch_geo3d(const ga_patch* pt, const double* ctrl, const double* const* w, int* bad,
                 hipStream_t st);
int launch_op2d(int mode, int nr, const ga_patch* pt, const double* x, double* y, double alpha,
                hipStream_t st, const double* gate = nullptr);
int launch_geo2d(const ga_patch* pt, const double* ctrl, const double* const* w, int* bad,
                 hipStream_t st);

void launch_fill(double* p, double v, size_t n, hipStream_t st);
// device-side control: gate = the CG scalars of right-hand side 0 (NSCAL per
// right-hand side); right-hand sides whose S_ACTIVE is 0 are left alone
void launch_fill_gated(int nr, double* y, size_t n, const double* gate, hipStream_t st);
bool pinv_band_fits(int dim, int p, const int* mf, size_t elem);
void launch_copy(double* dst, const double* src, size_t n, hipStream_t st);
void launch_scale_mul(double* out, const double* in, const double* s, int nr, size_t n, hipStream_t st);
void launch_gemm(int M, int N, int K, const double* X, long long ldx, long long sX,
                 const double* Y, long long ldy, long long sY, double* C, long long ldc,
                 long long sC, int batch, hipStream_t st);
bool pinv_axis_supported(int L);
template <typename S>
void launch_pinv_strided(const S* in, S* out, const S* A, int L, long long row_stride,
                         long long ncol, long long plane_stride, int planes_per_rhs,
                         long long n_free, int nr, const S* si, const S* so, hipStream_t st);
template <typename S>
void launch_pinv_contig(const S* in, S* out, const S* A, int L, long long nrows,
                        long long rows_per_rhs, long long n_free, const S* si, const S* so,
                        hipStream_t st);
// one patch of a multi-patch preconditioner pass.  Pass 0 (x axis, contiguous rows):
// p = {rows, rows per right-hand side}; passes 1-2 (strided): p = {row stride,
// columns per plane, plane stride, columns}.  Workgroup columns blk0 ..
struct PinvEntry {
  const void* A;              // the axis' inverse 1-D mass matrix (L x L)
  const void* si;             // scaling applied to the input, or null
  const void* so;             // scaling applied to the output, or null
  int L;
  long long p[4];
  long long off;              // segment offset in the batched vectors
  int blk0;
  int sys;                    // the patch's index in the batch
};
int pinv_ra_class(int L);
// dense per-axis preconditioner on the matrix cores (pinv_mfma.hip): the packed
// inverse of one axis for arithmetic `prec` (GA_FP64, GA_FP32 or GA_BF16), its size,
// and the three-pass application with the packed inverses apk[axis] (-1: an axis
// is too long)
bool pinv_mfma_supported(int prec, int L);
size_t pinv_mfma_pack_bytes(int prec, int L);
int pinv_mfma_pack(int prec, const double* A, int L, void* out, hipStream_t st);
int launch_pinv_mfma_f32(int prec, int dim, const int* mf, int nr, const float* r, float* z,
                         float* t0, float* t1, const void* const* apk, const float* s, long long n,
                         hipStream_t st);
int launch_pinv_mfma_f64(int dim, const int* mf, int nr, const double* r, double* z, double* t0,
                         double* t1, const void* const* apk, const double* s, long long n,
                         hipStream_t st);
// banded-Cholesky preconditioner (0 launched, 1 does not fit the LDS staging, -1 error)
// FP64 banded preconditioner whose last pass also sums r^T z per workgroup and, in
// the last workgroup per right-hand side, applies cgcg_gamma (3-D patches)
int launch_pinv_band_cgcg(int p, const int* mf, int nr, const double* r, double* z, double* t0,
                          double* t1, const double* const* cb, const double* s, long long n_free,
                          hipStream_t st, const double* gate, const CgFuse& f);
// Chronopoulos-Gear update of the active right-hand sides at iteration `it`: every
// workgroup sums the partials part_delta (RED_BLOCKS per right-hand side) of
// delta = z^T w, w = M z, and takes beta = gamma / gamma_prev, alpha = gamma /
// (delta - beta gamma / alpha_prev) (alpha = gamma / delta, p = z, s = w at it = 0);
// then p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s, w = 0.  Its first
// workgroup stores alpha and gamma for the next iteration and counts the iteration.
void launch_cgcg_update(int nr, int it, double* x, double* r, double* p, double* s, double* w,
                        const double* z, const double* part_delta, double* scal, size_t n,
                        hipStream_t st);
template <typename S>
int launch_pinv_band(int dim, int p, const int* mf, int nr, const S* r, S* z, S* t0, S* t1,
                     const S* const* cb, const S* s, long long n_free, hipStream_t st,
                     const double* gate = nullptr);
template <typename S>
void launch_pinv_group(int pass, int ra_class, const PinvEntry* ents, int nent, int nblk, int nr,
                       const S* in, S* out, long long stride, hipStream_t st,
                       BatchGate gate = BatchGate{nullptr, 0, 0});
void launch_scaling(double* s, const double* diagM, const double* dh0, const double* dh1,
                    const double* dh2, int mf0, int mf1, int mf2, hipStream_t st);
void launch_dot_partial(int nr, const double* a, const double* b, size_t n, double* part,
                        hipStream_t st, const double* gate = nullptr);
void launch_cg_start(int nr, const double* part_rz, const double* part_bn, double* scal,
                     double tol2, hipStream_t st);
void launch_cg_fallback(int nr, double* x, double* r, double* z, const double* b, const double* zb,
                        const double* scal, size_t n, hipStream_t st);
void launch_extrap(int k, int nh, const double* const* hist, double* X, size_t n, hipStream_t st);
void launch_cg_alpha(int nr, const double* part, double* scal, hipStream_t st);
void launch_cg_beta(int nr, const double* part, double* scal, hipStream_t st);
void launch_cg_xr(int nr, double* x, double* r, const double* p, const double* q,
                  const double* scal, size_t n, hipStream_t st);
void launch_cg_p(int nr, double* p, const double* z, const double* scal, size_t n, hipStream_t st);
void launch_predict(int k, double tau, StatePtrs sp, double* Y, size_t n, hipStream_t st);
void launch_predict_cz(int k, double tau, double cK, StatePtrs sp, double* Y, double* Z, size_t n,
                       hipStream_t st);
void launch_update(int k, double tau, Coefs c, StatePtrs sp, const double* X, size_t n,
                   hipStream_t st);
// one segment of n entries of batched vectors: the state pointers point at the
// segment, stage vectors are ys (xs) entries apart
void launch_predict_seg(int k, double tau, StatePtrs sp, double* Y, size_t n, size_t ys,
                        hipStream_t st);
void launch_update_seg(int k, double tau, Coefs c, StatePtrs sp, const double* X, size_t n,
                       size_t xs, hipStream_t st);
void launch_axpby(double* out, double a, const double* x, double b, const double* y, size_t n,
                  hipStream_t st);
// FP32 kernels of the mixed solve; with seg, system r covers entries
// seg[2r] .. seg[2r] + seg[2r+1] - 1 (n is then the longest system)
void launch_to_f32(float* o, const double* i, size_t n, hipStream_t st);
void launch_to_f64(double* o, const float* i, size_t n, hipStream_t st);
// BF16 bit patterns, rounded to nearest even
void launch_to_bf16(unsigned short* o, const double* i, size_t n, hipStream_t st);
void launch_add_f32(double* x, const float* d, size_t n, hipStream_t st);
void launch_fill_f32(float* p, size_t n, hipStream_t st);
void launch_copy_f32(float* d, const float* s, size_t n, hipStream_t st);
void launch_dot_ff(int nr, const float* a, const float* b, size_t n, double* part, hipStream_t st,
               const long long* seg = nullptr);
void launch_dot_df(int nr, const double* a, const float* b, size_t n, double* part, hipStream_t st,
               const long long* seg = nullptr);
void launch_dot2_f32(int nr, const float* r, const float* z, const float* q, size_t n, double* p1,
                     double* p2, hipStream_t st,
               const long long* seg = nullptr);
void launch_cg_beta_flex(int nr, const double* p1, const double* p2, double* scal, hipStream_t st);
// mixed-precision refinement: the outer test from rz = r^T P^{-1} r (partials; pass 0
// also sets b^T P^{-1} b from part_bn, or from rz with a zero guess, and the guess
// fallback flag) and the start of the inner PCG (scalars si) for the next pass
void launch_mx_outer(int nr, const double* part_rz, const double* part_bn, double* so, double* si,
                     double rtol2, double floor2, int pass, hipStream_t st);
// systems whose guess was rejected restart from zero: x = 0, r64 = b, r32 = b32, z32 = zb32
// accept inner solves the inner arithmetic resolves (nr <= 64), without an FP64 residual
void launch_mx_accept(int nr, double* so, const double* si, double floor2, hipStream_t st);
void launch_mx_fallback(int nr, double* x, double* r64, float* r32, float* z32, const double* b,
                        const float* b32, const float* zb32, const double* so, size_t n,
                        hipStream_t st);
void launch_cg_xr_f32(int nr, float* x, float* r, const float* p, const float* q,
                      const double* scal, size_t n, hipStream_t st,
               const long long* seg = nullptr);
void launch_cg_p_f32(int nr, float* p, const float* z, const double* scal, size_t n,
                     hipStream_t st,
               const long long* seg = nullptr);
void launch_sum_partials(int nr, const double* part, double* out, hipStream_t st);
// glued multi-patch: xl[j][i] = xg[j][map[i]]; yg[j][map[i]] += alpha yl[j][i] (atomic)
void launch_gather(int nr, const double* xg, long long Ng, const int* map, long long Nl, double* xl,
                   hipStream_t st);
void launch_scatter_add(int nr, const double* yl, long long Nl, const int* map, double alpha,
                        double* yg, long long Ng, hipStream_t st);
// segment-aware CG kernels: system s = entries seg[2s] .. seg[2s] + seg[2s+1] of each vector
void launch_dot_partial_seg(int ns, const double* a, const double* b, const long long* seg,
                            double* part, hipStream_t st);
void launch_cg_fallback_seg(int ns, double* x, double* r, double* z, const double* b,
                            const double* zb, const double* scal, const long long* seg,
                            size_t maxlen, hipStream_t st);
void launch_cg_xr_seg(int ns, double* x, double* r, const double* p, const double* q,
                      const double* scal, const long long* seg, size_t maxlen, hipStream_t st);
void launch_cg_p_seg(int ns, double* p, const double* z, const double* scal, const long long* seg,
                     size_t maxlen, hipStream_t st);

}  // namespace ga
