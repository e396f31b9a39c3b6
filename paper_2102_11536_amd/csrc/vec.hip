// Vector kernels of the solve and the time step: per-axis dense contractions
// of the Kronecker preconditioner, deterministic two-stage FP64 reductions,
// fused PCG updates, Taylor predictors and the 3k-vector state update.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ga {

namespace {

constexpr int VB = 256;  // threads per block of the streaming kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the block (VB threads = 4 waves); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < VB / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ void fill_k(double* p, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// y_r = 0 for the right-hand sides r = blockIdx.y that are still active
__global__ void fill_gated_k(double* y, size_t n, const double* __restrict__ gate) {
  const int r = blockIdx.y;
  if (gate[(size_t)r * NSCAL + S_ACTIVE] == 0.0) return;
  double* yr = y + (size_t)r * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    yr[i] = 0.0;
}

__global__ void copy_k(double* __restrict__ d, const double* __restrict__ s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

__global__ void axpby_k(double* out, double a, const double* x, double b, const double* y,
                        size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}

__global__ void scale_mul_k(double* out, const double* in, const double* __restrict__ s,
                            size_t n, size_t total) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = s[i % n] * in[i];
}

// C[b] = X[b] * Y[b], row-major, FP64; 64x64 output tile, 16-deep k chunks,
// 256 threads with a 4x4 register block each.
__global__ void __launch_bounds__(256)
gemm_f64_k(int M, int N, int K, const double* __restrict__ X, long long ldx, long long sX,
           const double* __restrict__ Y, long long ldy, long long sY, double* __restrict__ C,
           long long ldc, long long sC) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double Xs[BK][BM + 1];
  __shared__ double Ys[BK][BN + 1];
  const int b = blockIdx.z;
  const double* Xb = X + (size_t)b * sX;
  const double* Yb = Y + (size_t)b * sY;
  double* Cb = C + (size_t)b * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      int e = tid + l * 256;
      int r = e / BK, c = e % BK;  // X tile: row r, col c
      int gm = m0 + r, gk = k0 + c;
      Xs[c][r] = (gm < M && gk < K) ? Xb[(size_t)gm * ldx + gk] : 0.0;
      int r2 = e / BN, c2 = e % BN;  // Y tile: row r2 (k), col c2 (n)
      int gk2 = k0 + r2, gn = n0 + c2;
      Ys[r2][c2] = (gk2 < K && gn < N) ? Yb[(size_t)gk2 * ldy + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double xv[4], yv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = Xs[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) yv[j] = Ys[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += xv[i] * yv[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < M && gn < N) Cb[(size_t)gm * ldc + gn] = acc[i][j];
    }
}

__global__ void scaling_k(double* s, const double* __restrict__ d, const double* __restrict__ h0,
                          const double* __restrict__ h1, const double* __restrict__ h2, int mf0,
                          int mf1, int mf2) {
  const size_t n = (size_t)mf0 * mf1 * mf2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    int i0 = (int)(i % mf0), i1 = (int)((i / mf0) % mf1), i2 = (int)(i / ((size_t)mf0 * mf1));
    double dh = h0[i0] * h1[i1] * (h2 ? h2[i2] : 1.0);
    s[i] = sqrt(dh / d[i]);
  }
}

// part[r][block] = partial sum of a_r . b_r
__global__ void __launch_bounds__(VB)
dot_partial_k(const double* __restrict__ a, const double* __restrict__ b, size_t n,
              double* __restrict__ part, const double* __restrict__ gate) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.y;
  if (gate && gate[(size_t)r * NSCAL + S_ACTIVE] == 0.0) {   // converged: partial unused
    if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const double* ar = a + (size_t)r * n;
  const double* br = b + (size_t)r * n;
  double s = 0.0;
  // four points per trip with their loads in flight together; the additions keep the
  // point order of one point per trip, so the sum is bitwise the same
  const size_t stride = (size_t)gridDim.x * VB;
  size_t i = (size_t)blockIdx.x * VB + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = ar[i + u * stride];
      y[u] = br[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += x[u] * y[u];
  }
  for (; i < n; i += stride) s += ar[i] * br[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = s;
}

// the total of part[r][0 .. RED_BLOCKS-1] on every thread of the block (the same
// additions in the same order on each)
__device__ double sum_part_all(const double* part, int r, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += VB) v += part[(size_t)r * RED_BLOCKS + i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < VB / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

__device__ double sum_part(const double* part, int r, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += VB) v += part[(size_t)r * RED_BLOCKS + i];
  return block_sum(v, sh);
}

__global__ void __launch_bounds__(VB)
cg_start_k(const double* part_rz, const double* part_bn, double* scal, double tol2) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  double rz = sum_part(part_rz, r, sh);
  double bn = part_bn ? sum_part(part_bn, r, sh) : rz;
  if (threadIdx.x == 0) {
    double* s = scal + (size_t)r * NSCAL;
    // a nonzero initial guess is kept only if its preconditioned residual is
    // smaller than that of the zero guess (b itself); otherwise restart from zero
    s[S_RZ0] = rz;
    s[S_FALLBACK] = (part_bn && !(rz < bn)) ? 1.0 : 0.0;
    if (s[S_FALLBACK] != 0.0) rz = bn;
    s[S_RZ] = rz;
    s[S_BN2] = bn;
    s[S_TOL2] = tol2;
    s[S_ITERS] = 0.0;
    s[S_ALPHA] = 0.0;
    s[S_BETA] = 0.0;
    s[S_ACTIVE] = (bn > 0.0 && rz > tol2 * bn) ? 1.0 : 0.0;
  }
}

__global__ void __launch_bounds__(VB) cg_alpha_k(const double* part, double* scal) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  double pq = sum_part(part, r, sh);
  if (threadIdx.x == 0) {
    double* s = scal + (size_t)r * NSCAL;
    s[S_PQ] = pq;
    s[S_ALPHA] = (s[S_ACTIVE] != 0.0) ? s[S_RZ] / pq : 0.0;
  }
}

__global__ void __launch_bounds__(VB) cg_beta_k(const double* part, double* scal) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  double rz = sum_part(part, r, sh);
  if (threadIdx.x == 0) {
    double* s = scal + (size_t)r * NSCAL;
    if (s[S_ACTIVE] != 0.0) {
      s[S_BETA] = rz / s[S_RZ];
      s[S_RZ] = rz;
      s[S_ITERS] += 1.0;
      if (!(rz > s[S_TOL2] * s[S_BN2])) s[S_ACTIVE] = 0.0;
    } else {
      s[S_BETA] = 0.0;
    }
  }
}

__global__ void sum_partials_k(const double* part, double* out) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  double v = sum_part(part, r, sh);
  if (threadIdx.x == 0) out[r] = v;
}

__global__ void cg_fallback_k(double* __restrict__ x, double* __restrict__ r,
                              double* __restrict__ z, const double* __restrict__ b,
                              const double* __restrict__ zb, const double* __restrict__ scal,
                              size_t n) {
  const int rr = blockIdx.y;
  if (scal[(size_t)rr * NSCAL + S_FALLBACK] == 0.0) return;
  const size_t off = (size_t)rr * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    x[off + i] = 0.0;
    r[off + i] = b[off + i];
    z[off + i] = zb[off + i];
  }
}

// polynomial extrapolation of the stage solutions from their last nh values:
// X = sum_h c_h H_h with c = [1], [2,-1], [3,-3,1], [4,-6,4,-1] (newest first)
__global__ void extrap_k(int k, int nh, HistPtrs hp, double* __restrict__ X, size_t n) {
  const double c[4][4] = {{1, 0, 0, 0}, {2, -1, 0, 0}, {3, -3, 1, 0}, {4, -6, 4, -1}};
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    for (int j = 0; j < k; ++j) {
      double v = 0.0;
      for (int h = 0; h < nh; ++h) v += c[nh - 1][h] * hp.H[h * 4 + j][i];
      X[(size_t)j * n + i] = v;
    }
}

__global__ void cg_xr_k(double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ q,
                        const double* __restrict__ scal, size_t n) {
  const int rr = blockIdx.y;
  const double a = scal[(size_t)rr * NSCAL + S_ALPHA];
  if (a == 0.0) return;
  const size_t off = (size_t)rr * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    x[off + i] += a * p[off + i];
    r[off + i] -= a * q[off + i];
  }
}

// single-reduction PCG update of the active right-hand sides (see launch_cgcg_update)
__global__ void __launch_bounds__(VB)
cgcg_update_k(int it, double* __restrict__ x, double* __restrict__ r, double* __restrict__ p,
              double* __restrict__ s, double* __restrict__ w, const double* __restrict__ z,
              const double* __restrict__ part, double* __restrict__ scal, size_t n) {
  __shared__ double sh[VB / 64];
  const int rr = blockIdx.y;
  double* sc = scal + (size_t)rr * NSCAL;
  if (sc[S_ACTIVE] == 0.0) return;
  const double delta = sum_part_all(part, rr, sh);   // the same sum, in the same order, everywhere
  const int cur = it & 1, nxt = cur ^ 1;
  const double g = sc[S_RZ];
  const bool first = it == 0;
  const double beta = first ? 0.0 : g / sc[cur ? S_GPREV1 : S_GPREV0];
  const double a = first ? g / delta : g / (delta - beta * g / sc[cur ? S_ALPHA1 : S_ALPHA0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[nxt ? S_ALPHA1 : S_ALPHA0] = a;
    sc[nxt ? S_GPREV1 : S_GPREV0] = g;
    sc[S_ITERS] += 1.0;
  }
  const size_t off = (size_t)rr * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t k = off + i;
    const double zi = z[k], wi = w[k];
    const double pi = first ? zi : zi + beta * p[k];
    const double si = first ? wi : wi + beta * s[k];
    p[k] = pi;
    s[k] = si;
    x[k] += a * pi;
    r[k] -= a * si;
    w[k] = 0.0;
  }
}

__global__ void cg_p_k(double* __restrict__ p, const double* __restrict__ z,
                       const double* __restrict__ scal, size_t n) {
  const int rr = blockIdx.y;
  if (scal[(size_t)rr * NSCAL + S_ACTIVE] == 0.0) return;
  const double b = scal[(size_t)rr * NSCAL + S_BETA];
  const size_t off = (size_t)rr * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[off + i] = z[off + i] + b * p[off + i];
}

// Taylor predictor T_a = sum_{b=a..N} tau^{b-a}/(b-a)! L^b of slot s = a + 2
__device__ __forceinline__ double taylor(const double* Lv, int s, int ns, double tau) {
  double acc = 0.0, c = 1.0;
  for (int b = s; b < ns; ++b) {
    acc += c * Lv[b];
    c *= tau / (double)(b - s + 1);
  }
  return acc;
}

// Y[(j-1) * ys + i], i < n: the stage arguments (ys = n unless the entries are
// one segment of longer batched vectors)
__global__ void predict_k(int k, double tau, StatePtrs sp, double* __restrict__ Y, size_t n,
                          size_t ys) {
  const int ns = 3 * k;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double Lv[12];
    for (int s = 0; s < ns; ++s) Lv[s] = sp.L[s][i];
    for (int j = 1; j < k; ++j) Y[(size_t)(j - 1) * ys + i] = taylor(Lv, 3 * j - 3, ns, tau);
    Y[(size_t)(k - 1) * ys + i] = Lv[ns - 3];  // L^{N-2}
  }
}

// stage arguments with Rayleigh damping C = cM M + cK K: Y_j + cK Z_j (the
// stiffness argument of the combined K apply) and Z_j (the argument of C:
// T_{a_j-1} for j < k, L^{N-1} for j = k), Z written only if Zout is given
__global__ void predict_cz_k(int k, double tau, double cK, StatePtrs sp, double* __restrict__ Y,
                             double* __restrict__ Zout, size_t n) {
  const int ns = 3 * k;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double Lv[12];
    for (int s = 0; s < ns; ++s) Lv[s] = sp.L[s][i];
    for (int j = 1; j <= k; ++j) {
      const double y = j < k ? taylor(Lv, 3 * j - 3, ns, tau) : Lv[ns - 3];
      const double z = j < k ? taylor(Lv, 3 * j - 2, ns, tau) : Lv[ns - 2];
      Y[(size_t)(j - 1) * n + i] = y + cK * z;
      if (Zout) Zout[(size_t)(j - 1) * n + i] = z;
    }
  }
}

__global__ void update_k(int k, double tau, Coefs c, StatePtrs sp, const double* __restrict__ X,
                         size_t n, size_t xs) {
  const int ns = 3 * k;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double Lv[12];
    for (int s = 0; s < ns; ++s) Lv[s] = sp.L[s][i];
    for (int j = 1; j <= k; ++j) {
      const int sa = 3 * j - 1;  // slot of a_j = 3j-3
      const double Ta = taylor(Lv, sa, ns, tau);
      const double Ta1 = taylor(Lv, sa - 1, ns, tau);
      const double Ta2 = taylor(Lv, sa - 2, ns, tau);
      const double P = (X[(size_t)(j - 1) * xs + i] - Ta) / c.alpha[j - 1];
      sp.L[sa][i] = Ta + P;
      sp.L[sa - 1][i] = Ta1 + c.gamma[j - 1] * tau * P;
      sp.L[sa - 2][i] = Ta2 + c.beta[j - 1] * tau * tau * P;
    }
  }
}

// ---- segment-aware variants: system s occupies entries seg[2s] .. seg[2s] + seg[2s+1]
// of each vector (patches of a batch have different lengths)

__global__ void __launch_bounds__(VB)
dot_partial_seg_k(const double* __restrict__ a, const double* __restrict__ b,
                  const long long* __restrict__ seg, double* __restrict__ part) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.y;
  const size_t off = (size_t)seg[2 * r], n = (size_t)seg[2 * r + 1];
  double s = 0.0;
  // four points per trip with their loads in flight together, added in point order
  const size_t stride = (size_t)gridDim.x * VB;
  size_t i = (size_t)blockIdx.x * VB + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = a[off + i + u * stride];
      y[u] = b[off + i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += x[u] * y[u];
  }
  for (; i < n; i += stride) s += a[off + i] * b[off + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = s;
}

__global__ void cg_fallback_seg_k(double* __restrict__ x, double* __restrict__ r,
                                  double* __restrict__ z, const double* __restrict__ b,
                                  const double* __restrict__ zb, const double* __restrict__ scal,
                                  const long long* __restrict__ seg) {
  const int rr = blockIdx.y;
  if (scal[(size_t)rr * NSCAL + S_FALLBACK] == 0.0) return;
  const size_t off = (size_t)seg[2 * rr], n = (size_t)seg[2 * rr + 1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    x[off + i] = 0.0;
    r[off + i] = b[off + i];
    z[off + i] = zb[off + i];
  }
}

__global__ void cg_xr_seg_k(double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            const double* __restrict__ scal, const long long* __restrict__ seg) {
  const int rr = blockIdx.y;
  const double a = scal[(size_t)rr * NSCAL + S_ALPHA];
  if (a == 0.0) return;
  const size_t off = (size_t)seg[2 * rr], n = (size_t)seg[2 * rr + 1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    x[off + i] += a * p[off + i];
    r[off + i] -= a * q[off + i];
  }
}

__global__ void cg_p_seg_k(double* __restrict__ p, const double* __restrict__ z,
                           const double* __restrict__ scal, const long long* __restrict__ seg) {
  const int rr = blockIdx.y;
  if (scal[(size_t)rr * NSCAL + S_ACTIVE] == 0.0) return;
  const double b = scal[(size_t)rr * NSCAL + S_BETA];
  const size_t off = (size_t)seg[2 * rr], n = (size_t)seg[2 * rr + 1];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[off + i] = z[off + i] + b * p[off + i];
}

// glued multi-patch: local (patch-wise free) <-> global unknowns through the map
// G (local index -> global index), nr right-hand sides
__global__ void gather_k(int nr, const double* __restrict__ xg, long long Ng,
                         const int* __restrict__ map, long long Nl, double* __restrict__ xl) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nr * Nl;
       e += (long long)gridDim.x * blockDim.x) {
    const long long j = e / Nl, i = e % Nl;
    xl[e] = xg[j * Ng + map[i]];
  }
}

__global__ void scatter_add_k(int nr, const double* __restrict__ yl, long long Nl,
                              const int* __restrict__ map, double alpha, double* __restrict__ yg,
                              long long Ng) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nr * Nl;
       e += (long long)gridDim.x * blockDim.x) {
    const long long j = e / Nl, i = e % Nl;
    unsafeAtomicAdd(&yg[j * Ng + map[i]], alpha * yl[e]);
  }
}

inline unsigned nblocks(size_t n) {
  size_t b = (n + VB - 1) / VB;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void launch_fill(double* p, double v, size_t n, hipStream_t st) {
  if (n) hipLaunchKernelGGL(fill_k, dim3(nblocks(n)), dim3(VB), 0, st, p, v, n);
}
void launch_fill_gated(int nr, double* y, size_t n, const double* gate, hipStream_t st) {
  unsigned b = nblocks(n) > 2048 ? 2048 : nblocks(n);
  if (n) hipLaunchKernelGGL(fill_gated_k, dim3(b, nr), dim3(VB), 0, st, y, n, gate);
}
void launch_copy(double* d, const double* s, size_t n, hipStream_t st) {
  if (n) hipLaunchKernelGGL(copy_k, dim3(nblocks(n)), dim3(VB), 0, st, d, s, n);
}
void launch_axpby(double* out, double a, const double* x, double b, const double* y, size_t n,
                  hipStream_t st) {
  if (n) hipLaunchKernelGGL(axpby_k, dim3(nblocks(n)), dim3(VB), 0, st, out, a, x, b, y, n);
}
void launch_scale_mul(double* out, const double* in, const double* s, int nr, size_t n,
                      hipStream_t st) {
  size_t tot = (size_t)nr * n;
  hipLaunchKernelGGL(scale_mul_k, dim3(nblocks(tot)), dim3(VB), 0, st, out, in, s, n, tot);
}
void launch_gemm(int M, int N, int K, const double* X, long long ldx, long long sX,
                 const double* Y, long long ldy, long long sY, double* C, long long ldc,
                 long long sC, int batch, hipStream_t st) {
  dim3 grid((N + 63) / 64, (M + 63) / 64, batch);
  hipLaunchKernelGGL(gemm_f64_k, grid, dim3(256), 0, st, M, N, K, X, ldx, sX, Y, ldy, sY, C, ldc,
                     sC);
}
void launch_scaling(double* s, const double* d, const double* h0, const double* h1,
                    const double* h2, int mf0, int mf1, int mf2, hipStream_t st) {
  size_t n = (size_t)mf0 * mf1 * mf2;
  hipLaunchKernelGGL(scaling_k, dim3(nblocks(n)), dim3(VB), 0, st, s, d, h0, h1, h2, mf0, mf1,
                     mf2);
}
void launch_dot_partial(int nr, const double* a, const double* b, size_t n, double* part,
                        hipStream_t st, const double* gate) {
  hipLaunchKernelGGL(dot_partial_k, dim3(RED_BLOCKS, nr), dim3(VB), 0, st, a, b, n, part, gate);
}
void launch_gather(int nr, const double* xg, long long Ng, const int* map, long long Nl, double* xl,
                   hipStream_t st) {
  hipLaunchKernelGGL(gather_k, dim3(nblocks((size_t)nr * Nl)), dim3(VB), 0, st, nr, xg, Ng, map, Nl, xl);
}
void launch_scatter_add(int nr, const double* yl, long long Nl, const int* map, double alpha,
                        double* yg, long long Ng, hipStream_t st) {
  hipLaunchKernelGGL(scatter_add_k, dim3(nblocks((size_t)nr * Nl)), dim3(VB), 0, st, nr, yl, Nl, map,
                     alpha, yg, Ng);
}
void launch_dot_partial_seg(int ns, const double* a, const double* b, const long long* seg,
                            double* part, hipStream_t st) {
  hipLaunchKernelGGL(dot_partial_seg_k, dim3(RED_BLOCKS, ns), dim3(VB), 0, st, a, b, seg, part);
}
void launch_cg_fallback_seg(int ns, double* x, double* r, double* z, const double* b,
                            const double* zb, const double* scal, const long long* seg,
                            size_t maxlen, hipStream_t st) {
  unsigned bl = nblocks(maxlen) > 2048 ? 2048 : nblocks(maxlen);
  hipLaunchKernelGGL(cg_fallback_seg_k, dim3(bl, ns), dim3(VB), 0, st, x, r, z, b, zb, scal, seg);
}
void launch_cg_xr_seg(int ns, double* x, double* r, const double* p, const double* q,
                      const double* scal, const long long* seg, size_t maxlen, hipStream_t st) {
  unsigned bl = nblocks(maxlen) > 2048 ? 2048 : nblocks(maxlen);
  hipLaunchKernelGGL(cg_xr_seg_k, dim3(bl, ns), dim3(VB), 0, st, x, r, p, q, scal, seg);
}
void launch_cg_p_seg(int ns, double* p, const double* z, const double* scal, const long long* seg,
                     size_t maxlen, hipStream_t st) {
  unsigned bl = nblocks(maxlen) > 2048 ? 2048 : nblocks(maxlen);
  hipLaunchKernelGGL(cg_p_seg_k, dim3(bl, ns), dim3(VB), 0, st, p, z, scal, seg);
}
void launch_cg_start(int nr, const double* prz, const double* pbn, double* scal, double tol2,
                     hipStream_t st) {
  hipLaunchKernelGGL(cg_start_k, dim3(nr), dim3(VB), 0, st, prz, pbn, scal, tol2);
}
void launch_cg_fallback(int nr, double* x, double* r, double* z, const double* b, const double* zb,
                        const double* scal, size_t n, hipStream_t st) {
  unsigned bl = nblocks(n) > 2048 ? 2048 : nblocks(n);
  hipLaunchKernelGGL(cg_fallback_k, dim3(bl, nr), dim3(VB), 0, st, x, r, z, b, zb, scal, n);
}
void launch_extrap(int k, int nh, const double* const* hist, double* X, size_t n, hipStream_t st) {
  HistPtrs hp;
  for (int i = 0; i < 16; ++i) hp.H[i] = hist[i];
  hipLaunchKernelGGL(extrap_k, dim3(nblocks(n)), dim3(VB), 0, st, k, nh, hp, X, n);
}
void launch_cg_alpha(int nr, const double* part, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(cg_alpha_k, dim3(nr), dim3(VB), 0, st, part, scal);
}
void launch_cg_beta(int nr, const double* part, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(cg_beta_k, dim3(nr), dim3(VB), 0, st, part, scal);
}
void launch_sum_partials(int nr, const double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_partials_k, dim3(nr), dim3(VB), 0, st, part, out);
}
void launch_cg_xr(int nr, double* x, double* r, const double* p, const double* q,
                  const double* scal, size_t n, hipStream_t st) {
  unsigned b = nblocks(n) > 2048 ? 2048 : nblocks(n);
  hipLaunchKernelGGL(cg_xr_k, dim3(b, nr), dim3(VB), 0, st, x, r, p, q, scal, n);
}
void launch_cgcg_update(int nr, int it, double* x, double* r, double* p, double* s, double* w,
                        const double* z, const double* part_delta, double* scal, size_t n,
                        hipStream_t st) {
  unsigned b = nblocks(n) > 2048 ? 2048 : nblocks(n);
  hipLaunchKernelGGL(cgcg_update_k, dim3(b, nr), dim3(VB), 0, st, it, x, r, p, s, w, z, part_delta,
                     scal, n);
}
void launch_cg_p(int nr, double* p, const double* z, const double* scal, size_t n,
                 hipStream_t st) {
  unsigned b = nblocks(n) > 2048 ? 2048 : nblocks(n);
  hipLaunchKernelGGL(cg_p_k, dim3(b, nr), dim3(VB), 0, st, p, z, scal, n);
}
void launch_predict_cz(int k, double tau, double cK, StatePtrs sp, double* Y, double* Z, size_t n,
                       hipStream_t st) {
  hipLaunchKernelGGL(predict_cz_k, dim3(nblocks(n)), dim3(VB), 0, st, k, tau, cK, sp, Y, Z, n);
}
void launch_predict(int k, double tau, StatePtrs sp, double* Y, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(predict_k, dim3(nblocks(n)), dim3(VB), 0, st, k, tau, sp, Y, n, n);
}
void launch_update(int k, double tau, Coefs c, StatePtrs sp, const double* X, size_t n,
                   hipStream_t st) {
  hipLaunchKernelGGL(update_k, dim3(nblocks(n)), dim3(VB), 0, st, k, tau, c, sp, X, n, n);
}
void launch_predict_seg(int k, double tau, StatePtrs sp, double* Y, size_t n, size_t ys,
                        hipStream_t st) {
  if (n) hipLaunchKernelGGL(predict_k, dim3(nblocks(n)), dim3(VB), 0, st, k, tau, sp, Y, n, ys);
}
void launch_update_seg(int k, double tau, Coefs c, StatePtrs sp, const double* X, size_t n,
                       size_t xs, hipStream_t st) {
  if (n) hipLaunchKernelGGL(update_k, dim3(nblocks(n)), dim3(VB), 0, st, k, tau, c, sp, X, n, xs);
}

}  // namespace ga
