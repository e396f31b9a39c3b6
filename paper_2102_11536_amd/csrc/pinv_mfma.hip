// Kronecker preconditioner z = s * (Mz^-1 x My^-1 x Mx^-1)(s * r) (Sec. 5.4) as dense
// per-axis contractions on the matrix cores: along each tensor axis the lines of
// the vector are multiplied by the dense inverse A = Mhat_a^{-1} (L x L, symmetric)
// of the univariate parametric mass matrix.  Three arithmetic kinds:
//   BF16  v_mfma_f32_32x32x16_bf16: A and the vector entries rounded to BF16,
//         products accumulated in FP32 (FP32 vectors)
//   FP32  v_mfma_f32_32x32x2f32 (FP32 vectors and arithmetic)
//   FP64  v_mfma_f64_16x16x4f64 (FP64 vectors and arithmetic)
// A is packed once, per axis and kind, into the operand order of the instruction
// ("fragments"): fragment (kb, ib) lane l holds A[MM ib + l % MM][KK kb + KE (l / MM) + e]
// for e < KE (zero outside L).  Because A is symmetric the same fragments serve as
// the A operand (rows of A against columns of the vector) and as the B operand
// (rows of the vector against columns of A).
//   strided pass (y or z axis): a wave owns MM lines (consecutive in memory across
//     the axis), D[i][c] = sum_j A[i][j] v[c][j]; the line entries are the B operand,
//     read straight from the vector (the MM lanes of a half wave read consecutive
//     entries);
//   contiguous pass (x axis): a wave owns MM rows of the vector, staged in LDS with
//     coalesced loads, D[c][i] = sum_j v[c][j] A[j][i]; the rows are the A operand, so
//     the outputs of a lane group are consecutive entries of one row (coalesced stores).
// The input scaling s is folded into the first pass and the output scaling into the
// last one.  Every wave computes all L outputs of its lines (NB blocks of MM).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"

namespace ga {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int KIND> struct Mf;
// D layout of the 32 x 32 instructions: value v of lane l is row 8 (v / 4) + 4 (l / 32)
// + v % 4, column l % 32; of the 16 x 16 FP64 instruction: row l / 16 + 4 v, column l % 16
template <> struct Mf<GA_BF16> {
  using S = float;
  using Frag = bf16x8;
  using Acc = f32x16;
  static constexpr int MM = 32, KK = 16, KE = 8, NV = 16;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
  static __device__ __forceinline__ Frag frag(const S (&v)[KE]) {
    Frag f;
#pragma unroll
    for (int e = 0; e < KE; ++e) f[e] = (__bf16)v[e];
    return f;
  }
};
template <> struct Mf<GA_FP32> {
  using S = float;
  using Frag = float;
  using Acc = f32x16;
  static constexpr int MM = 32, KK = 2, KE = 1, NV = 16;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return 8 * (v >> 2) + 4 * (l >> 5) + (v & 3); }
  static __device__ __forceinline__ Frag frag(const S (&v)[KE]) { return v[0]; }
};
template <> struct Mf<GA_FP64> {
  using S = double;
  using Frag = double;
  using Acc = f64x4;
  static constexpr int MM = 16, KK = 4, KE = 1, NV = 4;
  static __device__ __forceinline__ Acc mma(Frag a, Frag b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int v, int l) { return (l >> 4) + 4 * v; }
  static __device__ __forceinline__ Frag frag(const S (&v)[KE]) { return v[0]; }
};

// fragment (kb, ib) of the packed inverse, nb blocks along the output axis
template <int KIND>
__global__ void pack_k(const double* __restrict__ A, int L, int kbn, int nb,
                       typename Mf<KIND>::Frag* __restrict__ out) {
  using M = Mf<KIND>;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)kbn * nb * 64) return;
  const int l = (int)(t % 64), f = (int)(t / 64), ib = f % nb, kb = f / nb;
  const int i = M::MM * ib + l % M::MM;
  typename M::S v[M::KE];
#pragma unroll
  for (int e = 0; e < M::KE; ++e) {
    const int j = M::KK * kb + M::KE * (l / M::MM) + e;
    v[e] = (i < L && j < L) ? (typename M::S)A[(size_t)i * L + j] : (typename M::S)0;
  }
  out[t] = M::frag(v);
}

__device__ __forceinline__ long long col_off(long long c, long long ncol, long long plane_stride) {
  return (c / ncol) * plane_stride + (c % ncol);
}

constexpr int WAVES = 4;

template <int KIND, int NB>
__global__ void __launch_bounds__(64 * WAVES)
pinv_mfma_strided_k(const typename Mf<KIND>::S* __restrict__ in, typename Mf<KIND>::S* __restrict__ out,
                    const typename Mf<KIND>::Frag* __restrict__ apk, int L, long long row_stride,
                    long long ncol, long long plane_stride, long long ncols_total, long long n_free,
                    const typename Mf<KIND>::S* __restrict__ si,
                    const typename Mf<KIND>::S* __restrict__ so) {
  using M = Mf<KIND>;
  using S = typename M::S;
  constexpr int MM = M::MM, KE = M::KE, KK = M::KK;
  constexpr int KBMAX = (MM * NB + KK - 1) / KK;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long cb = ((long long)blockIdx.x * WAVES + w) * MM;
  if (cb >= ncols_total) return;
  const S* inr = in + (size_t)blockIdx.y * n_free;
  S* outr = out + (size_t)blockIdx.y * n_free;
  const long long c = cb + lane % MM;
  const bool cok = c < ncols_total;
  const long long off = cok ? col_off(c, ncol, plane_stride) : 0;
  const int kbn = (L + KK - 1) / KK;
  // every entry of the lane's line it contributes, loaded up front
  S v[KBMAX][KE];
#pragma unroll
  for (int kb = 0; kb < KBMAX; ++kb)
#pragma unroll
    for (int e = 0; e < KE; ++e) {
      const int j = KK * kb + KE * (lane / MM) + e;
      S t = (S)0;
      if (cok && j < L) {
        const long long o = off + (long long)j * row_stride;
        t = inr[o];
        if (si) t *= si[o];
      }
      v[kb][e] = t;
    }
  typename M::Acc acc[NB];
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int q = 0; q < M::NV; ++q) acc[ib][q] = (S)0;
#pragma unroll
  for (int kb = 0; kb < KBMAX; ++kb) {
    if (kb < kbn) {
      const typename M::Frag b = M::frag(v[kb]);
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) acc[ib] = M::mma(apk[((size_t)kb * NB + ib) * 64 + lane], b, acc[ib]);
    }
  }
  if (!cok) return;
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int q = 0; q < M::NV; ++q) {
      const int i = MM * ib + M::row(q, lane);
      if (i < L) {
        const long long o = off + (long long)i * row_stride;
        outr[o] = so ? so[o] * (S)acc[ib][q] : (S)acc[ib][q];
      }
    }
}

template <int KIND, int NB>
__global__ void __launch_bounds__(64 * WAVES)
pinv_mfma_contig_k(const typename Mf<KIND>::S* __restrict__ in, typename Mf<KIND>::S* __restrict__ out,
                   const typename Mf<KIND>::Frag* __restrict__ apk, int L, long long nrows,
                   long long rows_per_rhs, long long n_free,
                   const typename Mf<KIND>::S* __restrict__ si,
                   const typename Mf<KIND>::S* __restrict__ so) {
  using M = Mf<KIND>;
  using S = typename M::S;
  constexpr int MM = M::MM, KE = M::KE, KK = M::KK;
  extern __shared__ unsigned char lds_raw[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kbn = (L + KK - 1) / KK;
  const int ldp = kbn * KK + 1;                 // padded LDS row (odd: no bank conflicts)
  S* tile = reinterpret_cast<S*>(lds_raw) + (size_t)w * MM * ldp;
  const long long r0 = ((long long)blockIdx.x * WAVES + w) * MM;
  // stage the wave's MM rows (zero beyond L and beyond the last row)
  for (int t = lane; t < MM * ldp; t += 64) {
    const int rr = t / ldp, j = t % ldp;
    const long long r = r0 + rr;
    S val = (S)0;
    if (r < nrows && j < L) {
      const long long lr = r % rows_per_rhs;
      val = in[(size_t)(r / rows_per_rhs) * n_free + lr * L + j];
      if (si) val *= si[lr * L + j];
    }
    tile[t] = val;
  }
  __syncthreads();
  if (r0 >= nrows) return;
  typename M::Acc acc[NB];
#pragma unroll
  for (int ib = 0; ib < NB; ++ib)
#pragma unroll
    for (int q = 0; q < M::NV; ++q) acc[ib][q] = (S)0;
  const S* trow = tile + (size_t)(lane % MM) * ldp + KE * (lane / MM);
#pragma unroll 2
  for (int kb = 0; kb < kbn; ++kb) {
    S v[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) v[e] = trow[KK * kb + e];
    const typename M::Frag a = M::frag(v);
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) acc[ib] = M::mma(a, apk[((size_t)kb * NB + ib) * 64 + lane], acc[ib]);
  }
#pragma unroll
  for (int q = 0; q < M::NV; ++q) {
    const long long r = r0 + M::row(q, lane);
    if (r >= nrows) continue;
    const long long lr = r % rows_per_rhs;
    const size_t ob = (size_t)(r / rows_per_rhs) * n_free + lr * L;
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      const int i = MM * ib + lane % MM;
      if (i < L) out[ob + i] = so ? so[lr * L + i] * (S)acc[ib][q] : (S)acc[ib][q];
    }
  }
}

template <int KIND>
int blocks_of(int L) { return (L + Mf<KIND>::MM - 1) / Mf<KIND>::MM; }

template <int KIND, int NB>
void strided_nb(const typename Mf<KIND>::S* in, typename Mf<KIND>::S* out, const void* apk, int L,
                long long row_stride, long long ncol, long long plane_stride, int planes_per_rhs,
                long long n_free, int nr, const typename Mf<KIND>::S* si,
                const typename Mf<KIND>::S* so, hipStream_t st) {
  constexpr int MM = Mf<KIND>::MM;
  const long long ncols_total = ncol * planes_per_rhs;
  const dim3 grid((unsigned)((ncols_total + WAVES * MM - 1) / (WAVES * MM)), (unsigned)nr);
  hipLaunchKernelGGL((pinv_mfma_strided_k<KIND, NB>), grid, dim3(64 * WAVES), 0, st, in, out,
                     (const typename Mf<KIND>::Frag*)apk, L, row_stride, ncol, plane_stride,
                     ncols_total, n_free, si, so);
}

template <int KIND, int NB>
void contig_nb(const typename Mf<KIND>::S* in, typename Mf<KIND>::S* out, const void* apk, int L,
               long long nrows, long long rows_per_rhs, long long n_free,
               const typename Mf<KIND>::S* si, const typename Mf<KIND>::S* so, hipStream_t st) {
  using M = Mf<KIND>;
  const int kbn = (L + M::KK - 1) / M::KK;
  const size_t lds = (size_t)WAVES * M::MM * (kbn * M::KK + 1) * sizeof(typename M::S);
  const dim3 grid((unsigned)((nrows + WAVES * M::MM - 1) / (WAVES * M::MM)));
  static size_t lds_set = 0;   // raise the dynamic LDS limit once per kernel instance
  if (lds > lds_set) {
    (void)hipFuncSetAttribute((const void*)pinv_mfma_contig_k<KIND, NB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    lds_set = lds;
  }
  hipLaunchKernelGGL((pinv_mfma_contig_k<KIND, NB>), grid, dim3(64 * WAVES), lds, st, in, out,
                     (const typename M::Frag*)apk, L, nrows, rows_per_rhs, n_free, si, so);
}

// NB (blocks along the axis) is a compile-time constant: 1..8 for the 32-wide
// kinds (L <= 256), 1..16 for FP64
template <int KIND>
int strided_any(const typename Mf<KIND>::S* in, typename Mf<KIND>::S* out, const void* apk, int L,
                long long rs, long long ncol, long long ps, int ppr, long long n_free, int nr,
                const typename Mf<KIND>::S* si, const typename Mf<KIND>::S* so, hipStream_t st) {
  switch (blocks_of<KIND>(L)) {
#define GA_S(NBV) case NBV: strided_nb<KIND, NBV>(in, out, apk, L, rs, ncol, ps, ppr, n_free, nr, si, so, st); return 0;
    GA_S(1) GA_S(2) GA_S(3) GA_S(4) GA_S(5) GA_S(6) GA_S(7) GA_S(8)
#undef GA_S
  }
  if constexpr (KIND == GA_FP64) {
    switch (blocks_of<KIND>(L)) {
#define GA_S(NBV) case NBV: strided_nb<KIND, NBV>(in, out, apk, L, rs, ncol, ps, ppr, n_free, nr, si, so, st); return 0;
      GA_S(9) GA_S(10) GA_S(11) GA_S(12) GA_S(13) GA_S(14) GA_S(15) GA_S(16)
#undef GA_S
    }
  }
  return -1;
}

template <int KIND>
int contig_any(const typename Mf<KIND>::S* in, typename Mf<KIND>::S* out, const void* apk, int L,
               long long nrows, long long rpr, long long n_free, const typename Mf<KIND>::S* si,
               const typename Mf<KIND>::S* so, hipStream_t st) {
  switch (blocks_of<KIND>(L)) {
#define GA_C(NBV) case NBV: contig_nb<KIND, NBV>(in, out, apk, L, nrows, rpr, n_free, si, so, st); return 0;
    GA_C(1) GA_C(2) GA_C(3) GA_C(4) GA_C(5) GA_C(6) GA_C(7) GA_C(8)
#undef GA_C
  }
  if constexpr (KIND == GA_FP64) {
    switch (blocks_of<KIND>(L)) {
#define GA_C(NBV) case NBV: contig_nb<KIND, NBV>(in, out, apk, L, nrows, rpr, n_free, si, so, st); return 0;
      GA_C(9) GA_C(10) GA_C(11) GA_C(12) GA_C(13) GA_C(14) GA_C(15) GA_C(16)
#undef GA_C
    }
  }
  return -1;
}

template <int KIND>
int apply_kind(int dim, const int* mf, int nr, const typename Mf<KIND>::S* r, typename Mf<KIND>::S* z,
               typename Mf<KIND>::S* t0, typename Mf<KIND>::S* t1, const void* const* apk,
               const typename Mf<KIND>::S* s, long long n, hipStream_t st) {
  const long long m0 = mf[0], m1 = mf[1], m2 = dim == 3 ? mf[2] : 1;
  int rc = contig_any<KIND>(r, t1, apk[0], (int)m0, nr * m1 * m2, m1 * m2, n, s, nullptr, st);
  if (rc) return rc;
  if (dim == 2)
    return strided_any<KIND>(t1, z, apk[1], (int)m1, m0, m0, 0, 1, n, nr, nullptr, s, st);
  rc = strided_any<KIND>(t1, t0, apk[1], (int)m1, m0, m0, m0 * m1, (int)m2, n, nr, nullptr, nullptr, st);
  if (rc) return rc;
  return strided_any<KIND>(t0, z, apk[2], (int)m2, m0 * m1, m0 * m1, 0, 1, n, nr, nullptr, s, st);
}

}  // namespace

bool pinv_mfma_supported(int prec, int L) {
  if (L < 1) return false;
  return prec == GA_FP64 ? L <= 256 : L <= 256;
}

size_t pinv_mfma_pack_bytes(int prec, int L) {
  auto sz = [&](int MM, int KK, size_t fb) {
    return (size_t)((L + KK - 1) / KK) * ((L + MM - 1) / MM) * 64 * fb;
  };
  if (prec == GA_BF16) return sz(32, 16, sizeof(bf16x8));
  if (prec == GA_FP32) return sz(32, 2, sizeof(float));
  return sz(16, 4, sizeof(double));
}

int pinv_mfma_pack(int prec, const double* A, int L, void* out, hipStream_t st) {
  if (!pinv_mfma_supported(prec, L)) return -1;
  auto launch = [&](auto kind_tag, int MM, int KK) {
    constexpr int K = decltype(kind_tag)::value;
    const int kbn = (L + KK - 1) / KK, nb = (L + MM - 1) / MM;
    const long long tot = (long long)kbn * nb * 64;
    hipLaunchKernelGGL(pack_k<K>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, L, kbn, nb,
                       (typename Mf<K>::Frag*)out);
  };
  if (prec == GA_BF16) launch(std::integral_constant<int, GA_BF16>(), 32, 16);
  else if (prec == GA_FP32) launch(std::integral_constant<int, GA_FP32>(), 32, 2);
  else launch(std::integral_constant<int, GA_FP64>(), 16, 4);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pinv_mfma_f32(int prec, int dim, const int* mf, int nr, const float* r, float* z,
                         float* t0, float* t1, const void* const* apk, const float* s, long long n,
                         hipStream_t st) {
  for (int a = 0; a < dim; ++a)
    if (!pinv_mfma_supported(prec, mf[a])) return -1;
  if (prec == GA_BF16) return apply_kind<GA_BF16>(dim, mf, nr, r, z, t0, t1, apk, s, n, st);
  if (prec == GA_FP32) return apply_kind<GA_FP32>(dim, mf, nr, r, z, t0, t1, apk, s, n, st);
  return -1;
}

int launch_pinv_mfma_f64(int dim, const int* mf, int nr, const double* r, double* z, double* t0,
                         double* t1, const void* const* apk, const double* s, long long n,
                         hipStream_t st) {
  for (int a = 0; a < dim; ++a)
    if (!pinv_mfma_supported(GA_FP64, mf[a])) return -1;
  return apply_kind<GA_FP64>(dim, mf, nr, r, z, t0, t1, apk, s, n, st);
}

}  // namespace ga
