// Kronecker preconditioner z = s * (Mz^-1 x My^-1 x Mx^-1)(s * r) (Sec. 5.4): one dense
// contraction per tensor axis with the symmetric inverse A = M_a^-1 of the univariate
// parametric mass matrix (free part, L x L), in FP64 on the vector ALU.
//
// Tiles match the axis length so nothing is wasted on ragged edges: a workgroup
// computes all L (<= 16*RA) outputs along the axis for 64 positions across it,
// 256 threads with a 9 x 4 (RA x 4) register tile each, the contraction staged in
// LDS 16 deep.  A is read row-wise (coalesced) thanks to its symmetry.
//   strided pass (y or z axis): out[c][i] = so * sum_j A[i][j] * si * in[c][j]
//     where column c runs over all planes of one vector (no per-plane raggedness)
//   contiguous pass (x axis):   out[r][i] = so * sum_j si * in[r][j] * A[j][i]
// The scaling s is folded into the first (si) and last (so) pass.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ga {

namespace {

constexpr int BK = 16;   // contraction depth per LDS stage
constexpr int BN = 64;   // positions across the axis per workgroup

// column c of one vector -> element offset of (j = 0, c)
__device__ __forceinline__ long long col_offset(long long c, long long ncol, long long plane_stride) {
  return (c / ncol) * plane_stride + (c % ncol);
}

// columns c0 .. c0+BN-1 of one right-hand side (inr, outr point at its first entry)
template <int RA, typename S>
__device__ __forceinline__ void
strided_body(const S* __restrict__ inr, S* __restrict__ outr,
             const S* __restrict__ A, int L, long long row_stride, long long ncol,
             long long plane_stride, long long ncols_total,
             const S* __restrict__ si, const S* __restrict__ so, long long c0) {
  constexpr int RP = 16 * RA;
  __shared__ S As[BK][RP + 1];
  __shared__ S Bs[BK][BN + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  // this thread's load slots in the B tile: (k = e / BN, column e % BN), e = tid + 256 l
  long long boff[BK * BN / 256];
  bool bok[BK * BN / 256];
#pragma unroll
  for (int l = 0; l < BK * BN / 256; ++l) {
    const long long c = c0 + (tid + 256 * l) % BN;
    bok[l] = c < ncols_total;
    boff[l] = bok[l] ? col_offset(c, ncol, plane_stride) : 0;
  }
  S acc[RA][4];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int j0 = 0; j0 < L; j0 += BK) {
    __syncthreads();
    for (int e = tid; e < BK * RP; e += 256) {
      const int k = e / RP, i = e % RP, j = j0 + k;
      As[k][i] = (i < L && j < L) ? A[(size_t)j * L + i] : (S)0;
    }
#pragma unroll
    for (int l = 0; l < BK * BN / 256; ++l) {
      const int e = tid + 256 * l, k = e / BN, cc = e % BN, j = j0 + k;
      S v = 0;
      if (bok[l] && j < L) {
        const long long off = boff[l] + (long long)j * row_stride;
        v = inr[off];
        if (si) v *= si[off];
      }
      Bs[k][cc] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      S av[RA], bv[4];
#pragma unroll
      for (int a = 0; a < RA; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const long long c = c0 + tx + 16 * b;
    if (c >= ncols_total) continue;
    const long long cb = col_offset(c, ncol, plane_stride);
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int i = ty + 16 * a;
      if (i < L) {
        const long long off = cb + (long long)i * row_stride;
        outr[off] = so ? so[off] * acc[a][b] : acc[a][b];
      }
    }
  }
}

template <int RA, typename S>
__global__ void __launch_bounds__(256)
pinv_strided_k(const S* __restrict__ in, S* __restrict__ out,
               const S* __restrict__ A, int L, long long row_stride, long long ncol,
               long long plane_stride, long long ncols_total, long long n_free,
               const S* __restrict__ si, const S* __restrict__ so) {
  strided_body<RA, S>(in + (size_t)blockIdx.y * n_free, out + (size_t)blockIdx.y * n_free, A, L,
                      row_stride, ncol, plane_stride, ncols_total, si, so,
                      (long long)blockIdx.x * BN);
}

// rows r0 .. r0+63 of all right-hand sides (row r of rhs r / rows_per_rhs)
template <int RA, typename S>
__device__ __forceinline__ void
contig_body(const S* __restrict__ in, S* __restrict__ out,
            const S* __restrict__ A, int L, long long nrows, long long rows_per_rhs,
            long long n_free, const S* __restrict__ si, const S* __restrict__ so, long long r0) {
  constexpr int RP = 16 * RA;
  constexpr int BM = 64;
  __shared__ S Xs[BK][BM + 1];
  __shared__ S As[BK][RP + 1];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  S acc[4][RA];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < RA; ++b) acc[a][b] = 0;
  for (int j0 = 0; j0 < L; j0 += BK) {
    __syncthreads();
    for (int e = tid; e < BK * RP; e += 256) {
      const int k = e / RP, i = e % RP, j = j0 + k;
      As[k][i] = (i < L && j < L) ? A[(size_t)j * L + i] : (S)0;
    }
#pragma unroll
    for (int l = 0; l < BK * BM / 256; ++l) {
      const int e = tid + 256 * l, rr = e / BK, k = e % BK, j = j0 + k;
      const long long r = r0 + rr;
      S v = 0;
      if (r < nrows && j < L) {
        const long long lr = r % rows_per_rhs;
        v = in[(size_t)(r / rows_per_rhs) * n_free + lr * L + j];
        if (si) v *= si[lr * L + j];
      }
      Xs[k][rr] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      S xv[4], av[RA];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = Xs[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < RA; ++b) av[b] = As[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < RA; ++b) acc[a][b] += xv[a] * av[b];
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const long long r = r0 + ty + 16 * a;
    if (r >= nrows) continue;
    const long long lr = r % rows_per_rhs;
    const size_t ob = (size_t)(r / rows_per_rhs) * n_free + lr * L;
#pragma unroll
    for (int b = 0; b < RA; ++b) {
      const int i = tx + 16 * b;
      if (i < L) out[ob + i] = so ? so[lr * L + i] * acc[a][b] : acc[a][b];
    }
  }
}

template <int RA, typename S>
__global__ void __launch_bounds__(256)
pinv_contig_k(const S* __restrict__ in, S* __restrict__ out,
              const S* __restrict__ A, int L, long long nrows, long long rows_per_rhs,
              long long n_free, const S* __restrict__ si, const S* __restrict__ so) {
  contig_body<RA, S>(in, out, A, L, nrows, rows_per_rhs, n_free, si, so, (long long)blockIdx.x * 64);
}

// several patches in one launch: workgroup column blockIdx.x belongs to the entry e
// with blk0 <= blockIdx.x < next blk0; blockIdx.y is the right-hand side
__device__ __forceinline__ int pinv_entry(const PinvEntry* ents, int nent) {
  int e = 0;
  while (e + 1 < nent && (int)blockIdx.x >= ents[e + 1].blk0) ++e;
  return e;
}

template <int RA, typename S>
__global__ void __launch_bounds__(256)
pinv_strided_group_k(const PinvEntry* __restrict__ ents, int nent, const S* __restrict__ in,
                     S* __restrict__ out, long long stride, BatchGate gate) {
  const PinvEntry& d = ents[pinv_entry(ents, nent)];
  if (!batch_active(gate, d.sys, blockIdx.y)) return;   // converged: the output is not used
  const size_t o = (size_t)d.off + (size_t)blockIdx.y * stride;
  strided_body<RA, S>(in + o, out + o, (const S*)d.A, d.L, d.p[0], d.p[1], d.p[2], d.p[3],
                      (const S*)d.si, (const S*)d.so, (long long)(blockIdx.x - d.blk0) * BN);
}

template <int RA, typename S>
__global__ void __launch_bounds__(256)
pinv_contig_group_k(const PinvEntry* __restrict__ ents, int nent, const S* __restrict__ in,
                    S* __restrict__ out, long long stride, BatchGate gate) {
  const PinvEntry& d = ents[pinv_entry(ents, nent)];
  if (gate.scal) {   // rows r0 .. r0+63 belong to right-hand sides r0 / rpr .. (r0+63) / rpr
    const long long r0 = (long long)(blockIdx.x - d.blk0) * 64;
    const long long last = min(r0 + 63, d.p[0] - 1);
    bool any = false;
    for (long long j = r0 / d.p[1]; j <= last / d.p[1]; ++j) any |= batch_active(gate, d.sys, (int)j);
    if (!any) return;
  }
  contig_body<RA, S>(in + d.off, out + d.off, (const S*)d.A, d.L, d.p[0], d.p[1], stride,
                     (const S*)d.si, (const S*)d.so, (long long)(blockIdx.x - d.blk0) * 64);
}

template <int RA, typename S>
void strided(const S* in, S* out, const S* A, int L, long long row_stride,
             long long ncol, long long plane_stride, int planes_per_rhs, long long n_free, int nr,
             const S* si, const S* so, hipStream_t st) {
  const long long ncols_total = ncol * planes_per_rhs;
  dim3 grid((unsigned)((ncols_total + BN - 1) / BN), (unsigned)nr);
  hipLaunchKernelGGL((pinv_strided_k<RA, S>), grid, dim3(256), 0, st, in, out, A, L, row_stride, ncol,
                     plane_stride, ncols_total, n_free, si, so);
}

template <int RA, typename S>
void contig(const S* in, S* out, const S* A, int L, long long nrows,
            long long rows_per_rhs, long long n_free, const S* si, const S* so,
            hipStream_t st) {
  hipLaunchKernelGGL((pinv_contig_k<RA, S>), dim3((unsigned)((nrows + 63) / 64)), dim3(256), 0, st, in,
                     out, A, L, nrows, rows_per_rhs, n_free, si, so);
}

}  // namespace

bool pinv_axis_supported(int L) { return L >= 1 && L <= 256; }

int pinv_ra_class(int L) { return L <= 64 ? 0 : (L <= 144 ? 1 : 2); }

template <typename S>
void launch_pinv_group(int pass, int ra_class, const PinvEntry* ents, int nent, int nblk, int nr,
                       const S* in, S* out, long long stride, hipStream_t st, BatchGate gate) {
  // pass 0 covers every right-hand side through its row index (p[0] = all rows)
  const dim3 grid((unsigned)nblk, pass == 0 ? 1u : (unsigned)nr);
#define GA_PG(RA)                                                                             \
  do {                                                                                        \
    if (pass == 0)                                                                            \
      hipLaunchKernelGGL((pinv_contig_group_k<RA, S>), grid, dim3(256), 0, st, ents, nent, in,  \
                         out, stride, gate);                                                  \
    else                                                                                      \
      hipLaunchKernelGGL((pinv_strided_group_k<RA, S>), grid, dim3(256), 0, st, ents, nent, in, \
                         out, stride, gate);                                                  \
  } while (0)
  if (ra_class == 0) GA_PG(4);
  else if (ra_class == 1) GA_PG(9);
  else GA_PG(16);
#undef GA_PG
}
template void launch_pinv_group<double>(int, int, const PinvEntry*, int, int, int, const double*,
                                        double*, long long, hipStream_t, BatchGate);
template void launch_pinv_group<float>(int, int, const PinvEntry*, int, int, int, const float*,
                                       float*, long long, hipStream_t, BatchGate);

template <typename S>
void launch_pinv_strided(const S* in, S* out, const S* A, int L, long long row_stride,
                         long long ncol, long long plane_stride, int planes_per_rhs,
                         long long n_free, int nr, const S* si, const S* so, hipStream_t st) {
  if (L <= 64) strided<4, S>(in, out, A, L, row_stride, ncol, plane_stride, planes_per_rhs, n_free, nr, si, so, st);
  else if (L <= 144) strided<9, S>(in, out, A, L, row_stride, ncol, plane_stride, planes_per_rhs, n_free, nr, si, so, st);
  else strided<16, S>(in, out, A, L, row_stride, ncol, plane_stride, planes_per_rhs, n_free, nr, si, so, st);
}

template <typename S>
void launch_pinv_contig(const S* in, S* out, const S* A, int L, long long nrows,
                        long long rows_per_rhs, long long n_free, const S* si, const S* so,
                        hipStream_t st) {
  if (L <= 64) contig<4, S>(in, out, A, L, nrows, rows_per_rhs, n_free, si, so, st);
  else if (L <= 144) contig<9, S>(in, out, A, L, nrows, rows_per_rhs, n_free, si, so, st);
  else contig<16, S>(in, out, A, L, nrows, rows_per_rhs, n_free, si, so, st);
}

template void launch_pinv_strided<double>(const double*, double*, const double*, int, long long,
                                          long long, long long, int, long long, int,
                                          const double*, const double*, hipStream_t);
template void launch_pinv_strided<float>(const float*, float*, const float*, int, long long,
                                         long long, long long, int, long long, int, const float*,
                                         const float*, hipStream_t);
template void launch_pinv_contig<double>(const double*, double*, const double*, int, long long,
                                         long long, long long, const double*, const double*,
                                         hipStream_t);
template void launch_pinv_contig<float>(const float*, float*, const float*, int, long long,
                                        long long, long long, const float*, const float*,
                                        hipStream_t);

}  // namespace ga
