// FP32 vector kernels of the mixed-precision mass solve: conversions between the
// FP64 outer iteration and the FP32 inner PCG, dot products accumulated in FP64,
// and the flexible (Polak-Ribiere) PCG updates of the inner solve.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ga {

namespace {

constexpr int VB = 256;

inline unsigned nb(size_t n) {
  size_t b = (n + VB - 1) / VB;
  if (b > 8192) b = 8192;
  return (unsigned)(b < 1 ? 1 : b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

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

__global__ void to_f32_k(float* __restrict__ o, const double* __restrict__ i, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB)
    o[k] = (float)i[k];
}

__global__ void to_f64_k(double* __restrict__ o, const float* __restrict__ i, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB)
    o[k] = (double)i[k];
}

// FP64 -> FP32 (nearest) -> BF16 (nearest even); NaN stays NaN
__global__ void to_bf16_k(unsigned short* __restrict__ o, const double* __restrict__ i, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB) {
    const unsigned u = __float_as_uint((float)i[k]);
    unsigned short h;
    if ((u & 0x7fffffffu) > 0x7f800000u) h = (unsigned short)((u >> 16) | 0x40u);
    else h = (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    o[k] = h;
  }
}

__global__ void add_f32_k(double* __restrict__ x, const float* __restrict__ d, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB)
    x[k] += (double)d[k];
}

__global__ void fill_f32_k(float* p, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB)
    p[k] = 0.0f;
}

__global__ void copy_f32_k(float* __restrict__ d, const float* __restrict__ s, size_t n) {
  for (size_t k = (size_t)blockIdx.x * VB + threadIdx.x; k < n; k += (size_t)gridDim.x * VB)
    d[k] = s[k];
}

// part[r][block] = sum a_r * b_r with FP64 accumulation (a, b FP32 or FP64)
// system r covers entries r*n .. r*n+n-1, or seg[2r] .. seg[2r]+seg[2r+1]-1 when a
// segment table is given (patches of a batch)
__device__ __forceinline__ void span(const long long* seg, int r, size_t n, size_t& off, size_t& len) {
  if (seg) {
    off = (size_t)seg[2 * r];
    len = (size_t)seg[2 * r + 1];
  } else {
    off = (size_t)r * n;
    len = n;
  }
}

template <typename TA, typename TB>
__global__ void __launch_bounds__(VB)
dotm_k(const TA* __restrict__ a, const TB* __restrict__ b, size_t n, double* __restrict__ part,
       const long long* __restrict__ seg) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.y;
  size_t off;
  span(seg, r, n, off, n);
  const TA* ar = a + off;
  const TB* br = b + off;
  double s = 0.0;
  // four points per trip with their loads in flight together, added in point order
  const size_t stride = (size_t)gridDim.x * VB;
  size_t i = (size_t)blockIdx.x * VB + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    TA x[4];
    TB y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = ar[i + u * stride];
      y[u] = br[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += (double)x[u] * (double)y[u];
  }
  for (; i < n; i += stride) s += (double)ar[i] * (double)br[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(size_t)r * gridDim.x + blockIdx.x] = s;
}

// two dots in one pass: r.z and z.q (FP32 vectors, FP64 accumulation)
__global__ void __launch_bounds__(VB)
dot2_k(const float* __restrict__ r, const float* __restrict__ z, const float* __restrict__ q,
       size_t n, double* __restrict__ p1, double* __restrict__ p2, const long long* __restrict__ seg) {
  __shared__ double sh[VB / 64];
  const int rr = blockIdx.y;
  size_t off;
  span(seg, rr, n, off, n);
  double s1 = 0.0, s2 = 0.0;
  // four points per trip with their loads in flight together, added in point order
  const size_t stride = (size_t)gridDim.x * VB;
  size_t i = (size_t)blockIdx.x * VB + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    float rv[4], zv[4], qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      rv[u] = r[off + i + u * stride];
      zv[u] = z[off + i + u * stride];
      qv[u] = q[off + i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double zd = zv[u];
      s1 += (double)rv[u] * zd;
      s2 += zd * (double)qv[u];
    }
  }
  for (; i < n; i += stride) {
    const double zv = z[off + i];
    s1 += (double)r[off + i] * zv;
    s2 += zv * (double)q[off + i];
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    p1[(size_t)rr * gridDim.x + blockIdx.x] = s1;
    p2[(size_t)rr * gridDim.x + blockIdx.x] = s2;
  }
}

__device__ double sum_part(const double* part, int r, double* sh) {
  double v = 0.0;
  for (int i = threadIdx.x; i < RED_BLOCKS; i += VB) v += part[(size_t)r * RED_BLOCKS + i];
  return block_sum(v, sh);
}

// flexible beta: rz_new = r.z, zq = z.q (q = M p), beta = -alpha zq / rz_old
__global__ void __launch_bounds__(VB) cg_beta_flex_k(const double* p1, const double* p2,
                                                     double* scal) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  const double rz = sum_part(p1, r, sh);
  const double zq = sum_part(p2, r, sh);
  if (threadIdx.x == 0) {
    double* s = scal + (size_t)r * NSCAL;
    if (s[S_ACTIVE] != 0.0) {
      s[S_BETA] = -s[S_ALPHA] * zq / s[S_RZ];
      s[S_RZ] = rz;
      s[S_ITERS] += 1.0;
      if (!(rz > s[S_TOL2] * s[S_BN2])) s[S_ACTIVE] = 0.0;
    } else {
      s[S_BETA] = 0.0;
    }
  }
}

// outer test and inner start of the mixed-precision refinement (one block per system)
__global__ void __launch_bounds__(VB)
mx_outer_k(const double* part_rz, const double* part_bn, double* so, double* si, double rtol2,
           double floor2, int pass) {
  __shared__ double sh[VB / 64];
  const int r = blockIdx.x;
  double rz = sum_part(part_rz, r, sh);
  const double bn = part_bn ? sum_part(part_bn, r, sh) : rz;
  if (threadIdx.x != 0) return;
  double* o = so + (size_t)r * NSCAL;
  double* in = si + (size_t)r * NSCAL;
  // a system that converged in an earlier pass, or whose inner result was accepted in
  // this one (o[11] < 0, set by mx_accept_k), keeps its scalars (its inner flags are
  // already off); only the per-pass iteration record is cleared or finished
  if (pass != 0 && o[S_ACTIVE] == 0.0) {
    if (o[11] < 0.0) {
      o[11] = 0.0;
    } else {
      o[10] = 0.0;
      o[11] = 0.0;
    }
    return;
  }
  if (pass == 0) {
    o[S_RZ0] = rz;
    o[S_FALLBACK] = (part_bn && !(rz < bn)) ? 1.0 : 0.0;   // keep a guess only if it beats zero
    if (o[S_FALLBACK] != 0.0) rz = bn;
    o[S_BN2] = bn;
    o[S_TOL2] = rtol2;
    o[S_ITERS] = 0.0;
    o[10] = 0.0;
    o[11] = 0.0;
  } else {
    o[S_ITERS] += in[S_ITERS];
    o[10] = in[S_ITERS];                                    // inner iterations of that pass
    o[11] = in[S_ACTIVE];                                   // still active when the pass ended
  }
  o[S_RZ] = rz;
  const double b2 = o[S_BN2];
  const bool active = b2 > 0.0 && rz > rtol2 * b2;
  o[S_ACTIVE] = active ? 1.0 : 0.0;
  // inner PCG for M d = r: stop at max(rtol_remaining / 2, floor) relative to |r|_P
  in[S_RZ] = rz;
  in[S_BN2] = rz;
  in[S_TOL2] = active ? fmax(0.25 * rtol2 * b2 / rz, floor2) : 1.0;
  in[S_ITERS] = 0.0;
  in[S_ALPHA] = 0.0;
  in[S_BETA] = 0.0;
  in[S_ACTIVE] = active ? 1.0 : 0.0;
}

// Acceptance of an inner solve without an FP64 residual (one thread per system): the
// inner PCG converged to at most half the outer tolerance, and the inner arithmetic's
// error, about floor |r|_P for the pass's starting residual r, is at most an eighth of
// it; the inner residual estimate then stands for the outer one
__global__ void mx_accept_k(int nr, double* so, const double* si, double floor2) {
  const int r = threadIdx.x;
  if (r >= nr) return;
  double* o = so + (size_t)r * NSCAL;
  const double* in = si + (size_t)r * NSCAL;
  if (o[S_ACTIVE] == 0.0 || in[S_ACTIVE] != 0.0) return;
  const double t2 = o[S_TOL2] * o[S_BN2];
  if (!(in[S_RZ] <= 0.25 * t2) || !(64.0 * floor2 * o[S_RZ] <= t2)) return;
  o[S_ITERS] += in[S_ITERS];
  o[10] = in[S_ITERS];   // inner iterations of this pass
  o[11] = -1.0;          // accepted in this pass (mx_outer_k turns it into 0: not cut)
  o[S_RZ] = in[S_RZ];
  o[S_ACTIVE] = 0.0;
}

__global__ void mx_fallback_k(double* __restrict__ x, double* __restrict__ r64, float* __restrict__ r32,
                              float* __restrict__ z32, const double* __restrict__ b,
                              const float* __restrict__ b32, const float* __restrict__ zb32,
                              const double* __restrict__ so, size_t n) {
  const int rr = blockIdx.y;
  if (so[(size_t)rr * NSCAL + S_FALLBACK] == 0.0) return;
  const size_t off = (size_t)rr * n;
  for (size_t i = (size_t)blockIdx.x * VB + threadIdx.x; i < n; i += (size_t)gridDim.x * VB) {
    x[off + i] = 0.0;
    r64[off + i] = b[off + i];
    r32[off + i] = b32[off + i];
    z32[off + i] = zb32[off + i];
  }
}

__global__ void cg_xr_f32_k(float* __restrict__ x, float* __restrict__ r,
                            const float* __restrict__ p, const float* __restrict__ q,
                            const double* __restrict__ scal, size_t n,
                            const long long* __restrict__ seg) {
  const int rr = blockIdx.y;
  const float a = (float)scal[(size_t)rr * NSCAL + S_ALPHA];
  if (a == 0.0f) return;
  size_t off;
  span(seg, rr, n, off, n);
  for (size_t i = (size_t)blockIdx.x * VB + threadIdx.x; i < n; i += (size_t)gridDim.x * VB) {
    x[off + i] += a * p[off + i];
    r[off + i] -= a * q[off + i];
  }
}

__global__ void cg_p_f32_k(float* __restrict__ p, const float* __restrict__ z,
                           const double* __restrict__ scal, size_t n,
                           const long long* __restrict__ seg) {
  const int rr = blockIdx.y;
  if (scal[(size_t)rr * NSCAL + S_ACTIVE] == 0.0) return;
  const float b = (float)scal[(size_t)rr * NSCAL + S_BETA];
  size_t off;
  span(seg, rr, n, off, n);
  for (size_t i = (size_t)blockIdx.x * VB + threadIdx.x; i < n; i += (size_t)gridDim.x * VB)
    p[off + i] = z[off + i] + b * p[off + i];
}

}  // namespace

void launch_to_f32(float* o, const double* i, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_k, dim3(nb(n)), dim3(VB), 0, st, o, i, n);
}
void launch_to_f64(double* o, const float* i, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_f64_k, dim3(nb(n)), dim3(VB), 0, st, o, i, n);
}
void launch_to_bf16(unsigned short* o, const double* i, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_bf16_k, dim3(nb(n)), dim3(VB), 0, st, o, i, n);
}
void launch_add_f32(double* x, const float* d, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(add_f32_k, dim3(nb(n)), dim3(VB), 0, st, x, d, n);
}
void launch_fill_f32(float* p, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(fill_f32_k, dim3(nb(n)), dim3(VB), 0, st, p, n);
}
void launch_copy_f32(float* d, const float* s, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_f32_k, dim3(nb(n)), dim3(VB), 0, st, d, s, n);
}
void launch_dot_ff(int nr, const float* a, const float* b, size_t n, double* part, hipStream_t st,
                   const long long* seg) {
  hipLaunchKernelGGL((dotm_k<float, float>), dim3(RED_BLOCKS, nr), dim3(VB), 0, st, a, b, n, part, seg);
}
void launch_dot_df(int nr, const double* a, const float* b, size_t n, double* part, hipStream_t st,
                   const long long* seg) {
  hipLaunchKernelGGL((dotm_k<double, float>), dim3(RED_BLOCKS, nr), dim3(VB), 0, st, a, b, n, part, seg);
}
void launch_dot2_f32(int nr, const float* r, const float* z, const float* q, size_t n, double* p1,
                     double* p2, hipStream_t st, const long long* seg) {
  hipLaunchKernelGGL(dot2_k, dim3(RED_BLOCKS, nr), dim3(VB), 0, st, r, z, q, n, p1, p2, seg);
}
void launch_cg_beta_flex(int nr, const double* p1, const double* p2, double* scal, hipStream_t st) {
  hipLaunchKernelGGL(cg_beta_flex_k, dim3(nr), dim3(VB), 0, st, p1, p2, scal);
}
void launch_mx_outer(int nr, const double* part_rz, const double* part_bn, double* so, double* si,
                     double rtol2, double floor2, int pass, hipStream_t st) {
  hipLaunchKernelGGL(mx_outer_k, dim3(nr), dim3(VB), 0, st, part_rz, part_bn, so, si, rtol2, floor2,
                     pass);
}
void launch_mx_accept(int nr, double* so, const double* si, double floor2, hipStream_t st) {
  hipLaunchKernelGGL(mx_accept_k, dim3(1), dim3(64), 0, st, nr, so, si, floor2);
}
void launch_mx_fallback(int nr, double* x, double* r64, float* r32, float* z32, const double* b,
                        const float* b32, const float* zb32, const double* so, size_t n,
                        hipStream_t st) {
  unsigned bl = nb(n) > 2048 ? 2048 : nb(n);
  hipLaunchKernelGGL(mx_fallback_k, dim3(bl, nr), dim3(VB), 0, st, x, r64, r32, z32, b, b32, zb32,
                     so, n);
}
void launch_cg_xr_f32(int nr, float* x, float* r, const float* p, const float* q,
                      const double* scal, size_t n, hipStream_t st, const long long* seg) {
  unsigned b = nb(n) > 2048 ? 2048 : nb(n);
  hipLaunchKernelGGL(cg_xr_f32_k, dim3(b, nr), dim3(VB), 0, st, x, r, p, q, scal, n, seg);
}
void launch_cg_p_f32(int nr, float* p, const float* z, const double* scal, size_t n,
                     hipStream_t st, const long long* seg) {
  unsigned b = nb(n) > 2048 ? 2048 : nb(n);
  hipLaunchKernelGGL(cg_p_f32_k, dim3(b, nr), dim3(VB), 0, st, p, z, scal, n, seg);
}

}  // namespace ga
