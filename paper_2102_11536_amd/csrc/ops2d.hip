// 2-D sum-factorised operator kernels (mass, stiffness, diag(M), geometry).
// One workgroup owns TE2 x TE2 elements; thread qx owns one column of Gauss
// points: x contraction and the whole y direction run in registers, the
// transposed x contraction through LDS, and the (TE2+p)^2 coefficient box is
// added to the output with FP64 atomics.  Factor layouts: W[tile][qy][qx],
// G[tile][qy][comp][qx] with comp = xx, xy, yy.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace ga {

template <int P>
struct Tile2 {
  static constexpr int Q = P + 1;
  static constexpr int TE = TE2;
  static constexpr int QT = TE * Q;
  static constexpr int NB = TE + P;
  static constexpr int TAB = TE * Q * (P + 1);
};

struct Geo2 {
  int n[2], m[2], mf[2], nt[2];
};

__device__ __forceinline__ long long free_index2(const Geo2& g, int i0, int i1) {
  int f0 = i0 - 1, f1 = i1 - 1;
  if (f0 < 0 || f1 < 0 || f0 >= g.mf[0] || f1 >= g.mf[1]) return -1;
  return (long long)f0 + (long long)g.mf[0] * f1;
}

template <int P, int MODE, int NR>
__global__ void __launch_bounds__(Tile2<P>::QT)
op2d_kernel(const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ fac,
            const double* __restrict__ tB0, const double* __restrict__ tB1,
            const double* __restrict__ tD0, const double* __restrict__ tD1, Geo2 g,
            long long n_free, double alpha, const double* __restrict__ gate) {
  // device-side control: nothing to do once all systems of the launch have converged
  if (gate) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) any |= gate[r * NSCAL + S_ACTIVE] != 0.0;
    if (!any) return;
  }
  using T = Tile2<P>;
  constexpr int Q = T::Q, QT = T::QT, NB = T::NB, TE = T::TE;
  __shared__ double sB[2][T::TAB];
  __shared__ double sD[2][T::TAB];
  __shared__ double xs[NR][NB * NB];
  __shared__ double S[NR][2][NB * QT];
  const int qx = threadIdx.x;
  const long long tile = blockIdx.x;
  const int tx = (int)(tile % g.nt[0]), ty = (int)(tile / g.nt[0]);
  const int e0x = tx * TE, e0y = ty * TE;
  for (int i = qx; i < T::TAB; i += QT) {
    sB[0][i] = tB0[(size_t)e0x * Q * (P + 1) + i];
    sB[1][i] = tB1[(size_t)e0y * Q * (P + 1) + i];
    sD[0][i] = tD0[(size_t)e0x * Q * (P + 1) + i];
    sD[1][i] = tD1[(size_t)e0y * Q * (P + 1) + i];
  }
  if (MODE != 2) {
    for (int i = qx; i < NR * NB * NB; i += QT) {
      int r = i / (NB * NB), b = i % (NB * NB);
      long long f = free_index2(g, e0x + b % NB, e0y + b / NB);
      xs[r][b] = (f >= 0) ? x[(size_t)r * n_free + f] : 0.0;
    }
  }
  __syncthreads();
  const int ex = qx / Q, jx = qx % Q;
  const double* bx = &sB[0][(ex * Q + jx) * (P + 1)];
  const double* dx = &sD[0][(ex * Q + jx) * (P + 1)];
  double a0[NR][NB], a1[NR][NB];
  if (MODE != 2) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int iy = 0; iy < NB; ++iy) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int a = 0; a <= P; ++a) {
          s0 += bx[a] * xs[r][iy * NB + ex + a];
          if (MODE == 1) s1 += dx[a] * xs[r][iy * NB + ex + a];
        }
        a0[r][iy] = s0;
        a1[r][iy] = s1;
      }
  }
  double sa[NR][NB], sb[NR][NB];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int iy = 0; iy < NB; ++iy) { sa[r][iy] = 0.0; sb[r][iy] = 0.0; }
  const double* ft = fac + (size_t)tile * QT * QT * (MODE == 1 ? 3 : 1);
#pragma unroll
  for (int ey = 0; ey < TE; ++ey)
#pragma unroll
    for (int jy = 0; jy < Q; ++jy) {
      const int qy = ey * Q + jy;
      const double* by = &sB[1][(ey * Q + jy) * (P + 1)];
      const double* dy = &sD[1][(ey * Q + jy) * (P + 1)];
      if (MODE == 1) {
        const double gxx = ft[((size_t)qy * 3 + 0) * QT + qx];
        const double gxy = ft[((size_t)qy * 3 + 1) * QT + qx];
        const double gyy = ft[((size_t)qy * 3 + 2) * QT + qx];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          double ux = 0.0, uy = 0.0;
#pragma unroll
          for (int b = 0; b <= P; ++b) {
            ux += by[b] * a1[r][ey + b];
            uy += dy[b] * a0[r][ey + b];
          }
          const double fx = gxx * ux + gxy * uy, fy = gxy * ux + gyy * uy;
#pragma unroll
          for (int b = 0; b <= P; ++b) {
            sa[r][ey + b] += by[b] * fx;  // pairs with Dx
            sb[r][ey + b] += dy[b] * fy;  // pairs with Bx
          }
        }
      } else {
        const double wq = ft[(size_t)qy * QT + qx];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          double u = 1.0;
          if (MODE == 0) {
            u = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) u += by[b] * a0[r][ey + b];
          }
          const double v = wq * u;
#pragma unroll
          for (int b = 0; b <= P; ++b) sa[r][ey + b] += by[b] * v;
        }
      }
    }
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int iy = 0; iy < NB; ++iy) {
      S[r][0][iy * QT + qx] = sa[r][iy];
      if (MODE == 1) S[r][1][iy * QT + qx] = sb[r][iy];
    }
  __syncthreads();
  for (int i = qx; i < NR * NB * NB; i += QT) {
    int r = i / (NB * NB), b = i % (NB * NB);
    int ix = b % NB, iy = b / NB;
    double acc = 0.0;
    for (int exx = 0; exx < TE; ++exx) {
      int a = ix - exx;
      if (a < 0 || a > P) continue;
      for (int j = 0; j < Q; ++j) {
        int q = exx * Q + j;
        if (MODE == 1)
          acc += sD[0][(exx * Q + j) * (P + 1) + a] * S[r][0][iy * QT + q] +
                 sB[0][(exx * Q + j) * (P + 1) + a] * S[r][1][iy * QT + q];
        else
          acc += sB[0][(exx * Q + j) * (P + 1) + a] * S[r][0][iy * QT + q];
      }
    }
    long long f = free_index2(g, e0x + ix, e0y + iy);
    if (f >= 0) unsafeAtomicAdd(&y[(size_t)r * n_free + f], alpha * acc);
  }
}

template <int P>
__global__ void __launch_bounds__(Tile2<P>::QT)
geo2d_kernel(const double* __restrict__ ctrl, const double* __restrict__ tB0,
             const double* __restrict__ tB1, const double* __restrict__ tD0,
             const double* __restrict__ tD1, const double* __restrict__ w0,
             const double* __restrict__ w1, Geo2 g, double* __restrict__ W,
             double* __restrict__ G, int* __restrict__ bad) {
  using T = Tile2<P>;
  constexpr int Q = T::Q, QT = T::QT, TE = T::TE;
  const int qx = threadIdx.x;
  const long long tile = blockIdx.x;
  const int tx = (int)(tile % g.nt[0]), ty = (int)(tile / g.nt[0]);
  const int ex = tx * TE + qx / Q, jx = qx % Q;
  const long long ndof = (long long)g.m[0] * g.m[1];
  for (int qy = 0; qy < QT; ++qy) {
    const int ey = ty * TE + qy / Q, jy = qy % Q;
    const size_t wi = (size_t)tile * QT * QT + (size_t)qy * QT + qx;
    const size_t gi = (size_t)tile * QT * QT * 3 + (size_t)qy * 3 * QT + qx;
    if (ex >= g.n[0] || ey >= g.n[1]) {
      W[wi] = 0.0;
      G[gi] = G[gi + QT] = G[gi + 2 * QT] = 0.0;
      continue;
    }
    const double* bx = &tB0[((size_t)ex * Q + jx) * (P + 1)];
    const double* dx = &tD0[((size_t)ex * Q + jx) * (P + 1)];
    const double* by = &tB1[((size_t)ey * Q + jy) * (P + 1)];
    const double* dy = &tD1[((size_t)ey * Q + jy) * (P + 1)];
    double J[2][2] = {{0, 0}, {0, 0}};
    for (int c1 = 0; c1 <= P; ++c1)
      for (int c0 = 0; c0 <= P; ++c0) {
        long long idx = (ex + c0) + (long long)g.m[0] * (ey + c1);
        for (int c = 0; c < 2; ++c) {
          double cp = ctrl[(size_t)c * ndof + idx];
          J[c][0] += cp * dx[c0] * by[c1];
          J[c][1] += cp * bx[c0] * dy[c1];
        }
      }
    const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    if (!(det > 0.0)) atomicOr(bad, 1);
    const double wq = w0[(size_t)ex * Q + jx] * w1[(size_t)ey * Q + jy];
    W[wi] = wq * det;
    // adj = [[J11, -J01], [-J10, J00]];  G = (w/det) adj adj^T
    const double a00 = J[1][1], a01 = -J[0][1], a10 = -J[1][0], a11 = J[0][0];
    const double sc = wq / det;
    G[gi] = sc * (a00 * a00 + a01 * a01);
    G[gi + QT] = sc * (a00 * a10 + a01 * a11);
    G[gi + 2 * QT] = sc * (a10 * a10 + a11 * a11);
  }
}

template <int P>
static int launch_op2d_p(int mode, int nr, const ga_patch* pt, const double* x, double* y,
                         double alpha, hipStream_t st, const double* gate) {
  Geo2 g;
  for (int a = 0; a < 2; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.nt[a] = pt->nt[a]; }
  const double* const* B = (mode == 2) ? pt->tabB2 : pt->tabB;
  const double* fac = (mode == 1) ? pt->G : pt->W;
  dim3 grid((unsigned)pt->n_tiles), block(Tile2<P>::QT);
#define GA_OP2(MODE, NRV)                                                                     \
  hipLaunchKernelGGL((op2d_kernel<P, MODE, NRV>), grid, block, 0, st, x, y, fac, B[0], B[1],   \
                     pt->tabD[0], pt->tabD[1], g, pt->n_free, alpha, gate)
  if (mode == 0) {
    if (nr == 1) GA_OP2(0, 1); else if (nr == 2) GA_OP2(0, 2); else GA_OP2(0, 3);
  } else if (mode == 1) {
    if (nr == 1) GA_OP2(1, 1); else if (nr == 2) GA_OP2(1, 2); else GA_OP2(1, 3);
  } else {
    GA_OP2(2, 1);
  }
#undef GA_OP2
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_op2d(int mode, int nr, const ga_patch* pt, const double* x, double* y, double alpha,
                hipStream_t st, const double* gate) {
  switch (pt->p) {
    case 1: return launch_op2d_p<1>(mode, nr, pt, x, y, alpha, st, gate);
    case 2: return launch_op2d_p<2>(mode, nr, pt, x, y, alpha, st, gate);
    case 3: return launch_op2d_p<3>(mode, nr, pt, x, y, alpha, st, gate);
    case 4: return launch_op2d_p<4>(mode, nr, pt, x, y, alpha, st, gate);
  }
  return -1;
}

int launch_geo2d(const ga_patch* pt, const double* ctrl, const double* const* w, int* bad,
                 hipStream_t st) {
  Geo2 g;
  for (int a = 0; a < 2; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.nt[a] = pt->nt[a]; }
#define GA_GEO2(PP)                                                                            \
  hipLaunchKernelGGL(geo2d_kernel<PP>, dim3((unsigned)pt->n_tiles), dim3(Tile2<PP>::QT), 0, st,  \
                     ctrl, pt->tabB[0], pt->tabB[1], pt->tabD[0], pt->tabD[1], w[0], w[1], g,    \
                     pt->W, pt->G, bad)
  switch (pt->p) {
    case 1: GA_GEO2(1); break;
    case 2: GA_GEO2(2); break;
    case 3: GA_GEO2(3); break;
    case 4: GA_GEO2(4); break;
    default: return -1;
  }
#undef GA_GEO2
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ga
