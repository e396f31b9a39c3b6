// Kronecker preconditioner z = s * (Mz^-1 x My^-1 x Mx^-1)(s * r) (Sec. 5.4) by banded
// Cholesky solves along each tensor axis instead of products with the dense inverses.
// The univariate mass matrix of degree p is banded (half-bandwidth p), and so is its
// Cholesky factor L: one forward and one backward substitution along a line of L
// coefficients costs about 4p + 2 flops per coefficient instead of the 2L of a dense
// product, so the preconditioner becomes a pure streaming operation.
//
//   row kernel (x axis): a workgroup of 256 threads stages 64 rows in LDS with
//     coalesced loads, 64 threads solve one row each, all threads store; the input
//     scaling s is fused into the load;
//   column kernel (y and z axes): one thread per line, streamed from and to global
//     memory (coalesced across a wave, 16 loads in flight per thread); the output
//     scaling is fused into the store of the last axis.
// Substitutions keep the last p results in registers (a sliding window).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace ga {

namespace {

// solve L L^T x = v along one line: v = src[i * stride], x -> dst[i * stride] (times
// so[i * stride] when so is given), i = 0 .. n-1; the forward result y is kept in dst.
// cb[i * (P+1)]: 1 / L(i,i); cb[i * (P+1) + d]: L(i, i-d); rows n .. n+P-1 are zero.
// Steps run in blocks of U: the U inputs and table rows are loaded first (indices
// clamped into range; results of steps past the end are dropped), so loads overlap
// and the only dependent chain is one multiply-add and one multiply per step.
template <int P, int U, typename S>
__device__ __forceinline__ void band_solve(const S* src, S* dst, long long stride, int n,
                                           const S* cb, const S* so, const S* rd = nullptr,
                                           S* rdot = nullptr) {
  constexpr int P1 = P + 1;
  S w[P];
#pragma unroll
  for (int d = 0; d < P; ++d) w[d] = 0;
  for (int i0 = 0; i0 < n; i0 += U) {      // L y = v, w[d] = y_{i-1-d}
    S vv[U], c[U][P1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = min(i0 + u, n - 1);
      vv[u] = src[i * stride];
#pragma unroll
      for (int d = 0; d <= P; ++d) c[u][d] = cb[i * P1 + d];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u < n) {
        S acc = vv[u];
#pragma unroll
        for (int d = P; d >= 1; --d) acc -= c[u][d] * w[d - 1];
        const S y = acc * c[u][0];
        vv[u] = y;
#pragma unroll
        for (int d = P - 1; d > 0; --d) w[d] = w[d - 1];
        w[0] = y;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u < n) dst[(i0 + u) * stride] = vv[u];
  }
#pragma unroll
  for (int d = 0; d < P; ++d) w[d] = 0;
  for (int i0 = n - 1; i0 >= 0; i0 -= U) {  // L^T x = y, w[d] = x_{i+1+d}
    S vv[U], c[U][P1], sc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = max(i0 - u, 0);
      vv[u] = dst[i * stride];
      sc[u] = (S)1;
      c[u][0] = cb[i * P1];
#pragma unroll
      for (int d = 1; d <= P; ++d) c[u][d] = cb[(i + d) * P1 + d];
    }
    if (so) {
#pragma unroll
      for (int u = 0; u < U; ++u) sc[u] = so[max(i0 - u, 0) * stride];
    }
    S rv[U];
    if (rd) {   // r at the same entries: sum r * z of the final values on the fly
#pragma unroll
      for (int u = 0; u < U; ++u) rv[u] = rd[max(i0 - u, 0) * stride];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 - u >= 0) {
        S acc = vv[u];
#pragma unroll
        for (int d = P; d >= 1; --d) acc -= c[u][d] * w[d - 1];
        const S x = acc * c[u][0];
        vv[u] = x * sc[u];
        if (rd) *rdot += rv[u] * vv[u];
#pragma unroll
        for (int d = P - 1; d > 0; --d) w[d] = w[d - 1];
        w[0] = x;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 - u >= 0) dst[(i0 - u) * stride] = vv[u];
  }
}

// copy n table entries to LDS with nthreads threads, 8 loads of each thread in flight
// before its stores (a wait per load would serialise the copy)
template <typename S>
__device__ __forceinline__ void copy_table(S* dst, const S* __restrict__ src, int n, int tid,
                                           int nthreads) {
  constexpr int K = 8;
  for (int e0 = 0; e0 < n; e0 += K * nthreads) {
    S v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = e0 + k * nthreads + tid;
      v[k] = e < n ? src[e] : (S)0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = e0 + k * nthreads + tid;
      if (e < n) dst[e] = v[k];
    }
  }
}

#ifndef GA_BAND_WT
#define GA_BAND_WT 256
#endif
#ifndef GA_BAND_NL
#define GA_BAND_NL 64
#endif
constexpr int WT = GA_BAND_WT;  // threads per workgroup: all stage and store, NL sweep
constexpr int NL = GA_BAND_NL;  // fewest lines per workgroup (one per sweeping thread)

// x axis: a workgroup stages nl consecutive rows (nl * L0 contiguous coefficients of
// one right-hand side) in LDS with coalesced loads by all WT threads, nl threads
// solve one row each, and all threads write the rows back; the input scaling si is
// fused into the load and the output scaling so (if given) into the store
template <int P, typename S>
__global__ void __launch_bounds__(WT)
band_row_k(const S* __restrict__ in, S* __restrict__ out, const S* __restrict__ cb0, int L0,
           long long rows, long long n_free, const S* __restrict__ si, const S* __restrict__ so,
           const double* __restrict__ gate, int nl) {
  // with a gate, a converged right-hand side (blockIdx.y) is skipped
  if (gate && gate[(size_t)blockIdx.y * NSCAL + S_ACTIVE] == 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  const int RS = L0 | 1;  // odd row stride
  S* pl = reinterpret_cast<S*>(smem_raw);
  S* c0 = pl + (size_t)nl * RS;              // factor table, (L0 + P) x (P + 1)
  const int tid = threadIdx.x;
  copy_table(c0, cb0, (L0 + P) * (P + 1), tid, WT);
  const long long r0 = (long long)blockIdx.x * nl;
  const int nrow = (int)min((long long)nl, rows - r0);
  const int cnt = nrow * L0;
  const long long base = r0 * L0;             // offset within one right-hand side
  const S* src = in + (size_t)blockIdx.y * n_free + base;
  S* dst = out + (size_t)blockIdx.y * n_free + base;
  constexpr int B = 8;
  for (int e0 = tid; e0 < cnt; e0 += WT * B) {
    S v[B], sv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = src[min(e0 + b * WT, cnt - 1)];
    if (si) {
#pragma unroll
      for (int b = 0; b < B; ++b) sv[b] = si[base + min(e0 + b * WT, cnt - 1)];
#pragma unroll
      for (int b = 0; b < B; ++b) v[b] *= sv[b];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int e = e0 + b * WT;
      if (e < cnt) pl[(e / L0) * RS + e % L0] = v[b];
    }
  }
  __syncthreads();
  if (tid < nrow) band_solve<P, 8, S>(pl + tid * RS, pl + tid * RS, 1, L0, c0, (const S*)nullptr);
  __syncthreads();
  for (int e0 = tid; e0 < cnt; e0 += WT * B) {
    S v[B], sv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int e = min(e0 + b * WT, cnt - 1);
      v[b] = pl[(e / L0) * RS + e % L0];
    }
    if (so) {
#pragma unroll
      for (int b = 0; b < B; ++b) sv[b] = so[base + min(e0 + b * WT, cnt - 1)];
#pragma unroll
      for (int b = 0; b < B; ++b) v[b] *= sv[b];
    }
#pragma unroll
    for (int b = 0; b < B; ++b)
      if (e0 + b * WT < cnt) dst[e0 + b * WT] = v[b];
  }
}

constexpr int CT = 64;  // threads (lines) per workgroup of the column kernel

// y or z axis: one thread per line, streamed from and to global memory (coalesced
// across the threads of a wave); line c starts at (c / per_plane) * plane_stride +
// c % per_plane and its L entries are `stride` apart.  The forward result is stored
// in the output and read back by the backward sweep; the output scaling so (if
// given) is fused into the final store.
template <int P, typename S>
__global__ void __launch_bounds__(CT)
band_col_k(const S* __restrict__ in, S* __restrict__ out, const S* __restrict__ cb,
           long long nlines, long long per_plane, long long plane_stride, long long stride, int L,
           long long n_free, const S* __restrict__ so, const double* __restrict__ gate) {
  if (gate && gate[(size_t)blockIdx.y * NSCAL + S_ACTIVE] == 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  S* ct = reinterpret_cast<S*>(smem_raw);       // factor table, (L + P) x (P + 1)
  const int lane = threadIdx.x;
  copy_table(ct, cb, (L + P) * (P + 1), lane, CT);
  __syncthreads();
  const long long c = (long long)blockIdx.x * CT + lane;
  if (c >= nlines) return;
  const long long o = (c / per_plane) * plane_stride + c % per_plane;
  band_solve<P, 16, S>(in + (size_t)blockIdx.y * n_free + o, out + (size_t)blockIdx.y * n_free + o,
                       stride, L, ct, so ? so + o : (const S*)nullptr);
}

// the z pass of the single-reduction PCG: as band_col_k (FP64, output scaling so),
// then each thread sums r * z over its line, and the workgroup partials of each
// right-hand side (blockIdx.y) are reduced by its last workgroup into gamma = r^T z
template <int P>
__global__ void __launch_bounds__(CT)
band_col_cg_k(const double* __restrict__ in, double* __restrict__ out, const double* __restrict__ cb,
              long long nlines, long long stride, int L, long long n_free,
              const double* __restrict__ so, const double* __restrict__ gate,
              const double* __restrict__ rr, CgFuse f) {
  if (gate && gate[(size_t)blockIdx.y * NSCAL + S_ACTIVE] == 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  double* ct = reinterpret_cast<double*>(smem_raw);   // factor table, (L + P) x (P + 1)
  __shared__ double sh[1];
  __shared__ int done;
  const int lane = threadIdx.x;
  copy_table(ct, cb, (L + P) * (P + 1), lane, CT);
  __syncthreads();
  const long long c = (long long)blockIdx.x * CT + lane;
  double acc = 0.0;
  if (c < nlines) {
    const size_t base = (size_t)blockIdx.y * n_free + c;   // lines of the z axis: per_plane = nlines
    band_solve<P, 16, double>(in + base, out + base, stride, L, ct, so + c, rr + base, &acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) f.part[(long long)blockIdx.y * f.pstride + blockIdx.x] = acc;
  CgFuse fy = f;
  fy.part = f.part + (long long)blockIdx.y * f.pstride;
  cgf_finish(fy, blockIdx.y, gridDim.x, 1, &done, sh,
             [&](int, double total) { cgcg_gamma(f.scal + (size_t)blockIdx.y * NSCAL, total); });
}

constexpr size_t LDS_MAX_BYTES = 152 * 1024;

int device_cus() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
  }
  return n;
}

size_t row_lds_bytes(int nl, long long L0, int p, size_t elem) {
  return ((size_t)nl * (L0 | 1) + (size_t)(L0 + p) * (p + 1)) * elem;
}

// rows per workgroup of the x pass: the fewest resident rounds of workgroups (LDS
// bounds the workgroups per CU), then the fewest rows (NL..WT, steps of 8); e.g. 72 for
// two FP64 right-hand sides at L0 = 129, where 64 leaves a second round of 10
int pick_nl(long long rows, int nr, long long L0, int p, size_t elem) {
  const long long slots_cu_lds = 160 * 1024;
  int best = NL;
  long long best_rounds = -1;
  for (int nl = NL; nl <= WT; nl += 8) {
    const size_t bytes = row_lds_bytes(nl, L0, p, elem);
    if (bytes > LDS_MAX_BYTES) break;
    const long long per_cu = std::max<long long>(1, slots_cu_lds / (long long)bytes);
    const long long nblk = (rows + nl - 1) / nl * nr;
    const long long rounds = (nblk + per_cu * device_cus() - 1) / (per_cu * device_cus());
    if (best_rounds < 0 || rounds < best_rounds) { best_rounds = rounds; best = nl; }
  }
  return best;
}

template <int P, typename S>
int launch_p(int dim, const int* mf, int nr, const S* r, S* z, S* t0, S* t1, const S* const* cb,
             const S* s, long long n_free, hipStream_t st, const double* gate) {
  const long long L0 = mf[0], L1 = mf[1], L2 = dim == 3 ? mf[2] : 1;
  const long long rows = L1 * L2;
  const int nl = pick_nl(rows, nr, L0, P, sizeof(S));
  const size_t row_bytes = row_lds_bytes(nl, L0, P, sizeof(S));
  const long long Lc = std::max(L1, L2);
  const size_t col_bytes = (size_t)(Lc + P) * (P + 1) * sizeof(S);
  if (row_bytes > LDS_MAX_BYTES || col_bytes > LDS_MAX_BYTES) return 1;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&band_row_k<P, S>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX_BYTES);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&band_col_k<P, S>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX_BYTES);
    attr = true;
  }
  // x: r -> t1 (input scaling)
  hipLaunchKernelGGL((band_row_k<P, S>), dim3((unsigned)((rows + nl - 1) / nl), nr), dim3(WT),
                     row_bytes, st, r, t1, cb[0], (int)L0, rows, n_free, s, (const S*)nullptr, gate,
                     nl);
  // y: t1 -> (3-D: t0; 2-D: z with the output scaling)
  const long long ny = L0 * L2;
  hipLaunchKernelGGL((band_col_k<P, S>), dim3((unsigned)((ny + CT - 1) / CT), nr), dim3(CT),
                     (size_t)(L1 + P) * (P + 1) * sizeof(S), st, t1,
                     dim == 3 ? t0 : z, cb[1], ny, L0, L0 * L1, L0, (int)L1, n_free,
                     dim == 3 ? (const S*)nullptr : s, gate);
  if (dim == 3) {
    // z: t0 -> z (output scaling)
    const long long nz = L0 * L1;
    hipLaunchKernelGGL((band_col_k<P, S>), dim3((unsigned)((nz + CT - 1) / CT), nr), dim3(CT),
                       (size_t)(L2 + P) * (P + 1) * sizeof(S), st, t0, z, cb[2],
                       nz, nz, 0LL, nz, (int)L2, n_free, s, gate);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

// 0: launched; 1: the rows do not fit the LDS staging (use the dense passes);
// -1: launch error.  t0, t1: scratch vectors like z.
template <typename S>
int launch_pinv_band(int dim, int p, const int* mf, int nr, const S* r, S* z, S* t0, S* t1,
                     const S* const* cb, const S* s, long long n_free, hipStream_t st,
                     const double* gate) {
  switch (p) {
    case 1: return launch_p<1, S>(dim, mf, nr, r, z, t0, t1, cb, s, n_free, st, gate);
    case 2: return launch_p<2, S>(dim, mf, nr, r, z, t0, t1, cb, s, n_free, st, gate);
    case 3: return launch_p<3, S>(dim, mf, nr, r, z, t0, t1, cb, s, n_free, st, gate);
    case 4: return launch_p<4, S>(dim, mf, nr, r, z, t0, t1, cb, s, n_free, st, gate);
  }
  return 1;
}

bool pinv_band_fits(int dim, int p, const int* mf, size_t elem) {
  if (p < 1 || p > 4) return false;
  const long long L0 = mf[0], L1 = mf[1], L2 = dim == 3 ? mf[2] : 1;
  const size_t row_bytes = ((size_t)NL * (L0 | 1) + (size_t)(L0 + p) * (p + 1)) * elem;
  const size_t col_bytes = (size_t)(std::max(L1, L2) + p) * (p + 1) * elem;
  return row_bytes <= LDS_MAX_BYTES && col_bytes <= LDS_MAX_BYTES;
}

namespace {
template <int P>
int band_cgcg_p(const int* mf, int nr, const double* r, double* z, double* t0, double* t1,
                const double* const* cb, const double* s, long long n_free, hipStream_t st,
                const double* gate, const CgFuse& f) {
  const long long L0 = mf[0], L1 = mf[1], L2 = mf[2];
  const long long rows = L1 * L2;
  const int nl = pick_nl(rows, nr, L0, P, sizeof(double));
  const size_t row_bytes = row_lds_bytes(nl, L0, P, sizeof(double));
  const size_t col_bytes = (size_t)(std::max(L1, L2) + P) * (P + 1) * sizeof(double);
  if (row_bytes > LDS_MAX_BYTES || col_bytes > LDS_MAX_BYTES) return 1;
  const long long nz = L0 * L1;
  if ((nz + CT - 1) / CT > f.pstride || nr > CGF_MAXRHS) return 1;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(&band_row_k<P, double>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX_BYTES);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&band_col_k<P, double>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX_BYTES);
    hipFuncSetAttribute(reinterpret_cast<const void*>(&band_col_cg_k<P>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX_BYTES);
    attr = true;
  }
  hipLaunchKernelGGL((band_row_k<P, double>), dim3((unsigned)((rows + nl - 1) / nl), nr), dim3(WT),
                     row_bytes, st, r, t1, cb[0], (int)L0, rows, n_free, s, (const double*)nullptr,
                     gate, nl);
  const long long ny = L0 * L2;
  hipLaunchKernelGGL((band_col_k<P, double>), dim3((unsigned)((ny + CT - 1) / CT), nr), dim3(CT),
                     (size_t)(L1 + P) * (P + 1) * sizeof(double), st, t1, t0, cb[1], ny, L0, L0 * L1,
                     L0, (int)L1, n_free, (const double*)nullptr, gate);
  hipLaunchKernelGGL((band_col_cg_k<P>), dim3((unsigned)((nz + CT - 1) / CT), nr), dim3(CT),
                     (size_t)(L2 + P) * (P + 1) * sizeof(double), st, t0, z, cb[2], nz, nz, (int)L2,
                     n_free, s, gate, r, f);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace

int launch_pinv_band_cgcg(int p, const int* mf, int nr, const double* r, double* z, double* t0,
                          double* t1, const double* const* cb, const double* s, long long n_free,
                          hipStream_t st, const double* gate, const CgFuse& f) {
  switch (p) {
    case 1: return band_cgcg_p<1>(mf, nr, r, z, t0, t1, cb, s, n_free, st, gate, f);
    case 2: return band_cgcg_p<2>(mf, nr, r, z, t0, t1, cb, s, n_free, st, gate, f);
    case 3: return band_cgcg_p<3>(mf, nr, r, z, t0, t1, cb, s, n_free, st, gate, f);
    case 4: return band_cgcg_p<4>(mf, nr, r, z, t0, t1, cb, s, n_free, st, gate, f);
  }
  return 1;
}

template int launch_pinv_band<double>(int, int, const int*, int, const double*, double*, double*,
                                      double*, const double* const*, const double*, long long,
                                      hipStream_t, const double*);
template int launch_pinv_band<float>(int, int, const int*, int, const float*, float*, float*,
                                     float*, const float* const*, const float*, long long,
                                     hipStream_t, const double*);

}  // namespace ga
