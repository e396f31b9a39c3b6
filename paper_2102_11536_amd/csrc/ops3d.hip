// 3-D sum-factorised operator kernels for gfx950.
//
//   y += alpha * B^T diag(W) B x                        (mass, eq. mass_matrix)
//   y += alpha * sum_ab D_a^T diag(G_ab) D_b x           (stiffness, K of eq. mp)
//   y  = (B o B)^T W                                     (diag(M), the D of Sec. 5.4)
//
// with B = Bz (x) By (x) Bx the tensor basis at the Gauss points and
// W = w|det J|, G = w|det J| J^{-1} J^{-T} stored per quadrature point.
//
// One workgroup owns a tile of TE^3 elements; its (TE*Q)^2 threads each own
// one (qx, qy) column of Gauss points through the tile's z extent (Q = p+1
// points per element).  Per tile: the (TE+p)^3 coefficient box is staged in
// LDS, contracted along x in LDS, along y and z in registers; the factor
// stream (W or G) is read once, coalesced, in the tile-major layout written
// by the setup kernel; the transposed contractions run back z (registers),
// y and x (LDS, plane by plane), and the box is added to the output with
// FP64 atomics (neighbouring tiles share p coefficient layers).
#include <hip/hip_runtime.h>

#include "ga_internal.h"
#include "kernels.h"

namespace ga {

template <int P>
struct Tile3 {
  static constexpr int Q = P + 1;
  static constexpr int TE = TE3;
  static constexpr int QT = TE * Q;      // Gauss points per tile edge
  static constexpr int NB = TE + P;      // coefficients per tile edge
  static constexpr int NT = QT * QT;     // threads per workgroup
  static constexpr int TAB = TE * Q * (P + 1);
};

struct Geo3 {
  int n[3], m[3], mf[3], nt[3];
};

// index of a full-grid coefficient (i0,i1,i2) in the free vector, or -1
__device__ __forceinline__ long long free_index3(const Geo3& g, int i0, int i1, int i2) {
  int f0 = i0 - 1, f1 = i1 - 1, f2 = i2 - 1;
  if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= g.mf[0] || f1 >= g.mf[1] || f2 >= g.mf[2]) return -1;
  return (long long)f0 + (long long)g.mf[0] * (f1 + (long long)g.mf[1] * f2);
}

// MODE: 0 mass, 1 stiffness, 2 diag(M) (tables hold squared values, x unused)
template <int P, int MODE, int NR>
__global__ void __launch_bounds__(Tile3<P>::NT)
op3d_kernel(const double* __restrict__ x, double* __restrict__ y,
            const double* __restrict__ fac,
            const double* __restrict__ tB0, const double* __restrict__ tB1,
            const double* __restrict__ tB2, const double* __restrict__ tD0,
            const double* __restrict__ tD1, const double* __restrict__ tD2,
            Geo3 g, long long n_free, double alpha) {
  using T = Tile3<P>;
  constexpr int Q = T::Q, QT = T::QT, NB = T::NB, NT = T::NT, TE = T::TE;
  constexpr int NPL = NB * NB;                  // coefficients per box plane
  constexpr int NA = (MODE == 1) ? 2 : 1;       // x-contracted fields
  constexpr int NG = (MODE == 1) ? 3 : 1;       // fields at Gauss points
  constexpr int FWD = NB * NB * NB + NA * NB * NB * QT;
  constexpr int BWD = NG * QT * QT + 2 * NB * QT;
  constexpr int WORK = (FWD > BWD ? FWD : BWD);

  __shared__ double sB[3][T::TAB];
  __shared__ double sD[3][T::TAB];
  __shared__ double work[NR][WORK];

  const int tid = threadIdx.x;
  const int qx = tid % QT, qy = tid / QT;
  const long long tile = blockIdx.x;
  const int tx = (int)(tile % g.nt[0]);
  const int ty = (int)((tile / g.nt[0]) % g.nt[1]);
  const int tz = (int)(tile / ((long long)g.nt[0] * g.nt[1]));
  const int e0[3] = {tx * TE, ty * TE, tz * TE};

  // element tables of this tile
  for (int i = tid; i < T::TAB; i += NT) {
    sB[0][i] = tB0[(size_t)e0[0] * Q * (P + 1) + i];
    sB[1][i] = tB1[(size_t)e0[1] * Q * (P + 1) + i];
    sB[2][i] = tB2[(size_t)e0[2] * Q * (P + 1) + i];
    if (MODE == 1) {
      sD[0][i] = tD0[(size_t)e0[0] * Q * (P + 1) + i];
      sD[1][i] = tD1[(size_t)e0[1] * Q * (P + 1) + i];
      sD[2][i] = tD2[(size_t)e0[2] * Q * (P + 1) + i];
    }
  }

  __syncthreads();
  const int eyq = qy / Q, jyq = qy % Q;

  // ---- forward: box -> (qx, qy, iz) values in registers ----
  double c0[NR][NB], cx[NR][NB], cy[NR][NB];
  if (MODE != 2) {
    for (int i = tid; i < NR * NB * NPL; i += NT) {
      int r = i / (NB * NPL), b = i % (NB * NPL);
      int ix = b % NB, iy = (b / NB) % NB, iz = b / NPL;
      long long f = free_index3(g, e0[0] + ix, e0[1] + iy, e0[2] + iz);
      work[r][b] = (f >= 0) ? x[(size_t)r * n_free + f] : 0.0;
    }
    __syncthreads();
    // x contraction: A[r][a][iz][iy][qx]
    for (int i = tid; i < NR * NB * NB * QT; i += NT) {
      int r = i / (NB * NB * QT), b = i % (NB * NB * QT);
      int q = b % QT, iy = (b / QT) % NB, iz = b / (QT * NB);
      int ex = q / Q, jx = q % Q;
      const double* bv = &sB[0][(ex * Q + jx) * (P + 1)];
      const double* xs = &work[r][iz * NPL + iy * NB + ex];
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int a = 0; a <= P; ++a) s0 += bv[a] * xs[a];
      if (MODE == 1) {
        const double* dv = &sD[0][(ex * Q + jx) * (P + 1)];
#pragma unroll
        for (int a = 0; a <= P; ++a) s1 += dv[a] * xs[a];
      }
      double* A = &work[r][NB * NPL];
      A[b] = s0;
      if (MODE == 1) A[NB * NB * QT + b] = s1;
    }
    __syncthreads();
    // y contraction in registers
    const double* by = &sB[1][(eyq * Q + jyq) * (P + 1)];
    const double* dy = &sD[1][(eyq * Q + jyq) * (P + 1)];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double* A0 = &work[r][NB * NPL];
      const double* A1 = A0 + NB * NB * QT;
#pragma unroll
      for (int iz = 0; iz < NB; ++iz) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) {
          double a0 = A0[(iz * NB + eyq + b) * QT + qx];
          s0 += by[b] * a0;
          if (MODE == 1) {
            s1 += by[b] * A1[(iz * NB + eyq + b) * QT + qx];
            s2 += dy[b] * a0;
          }
        }
        c0[r][iz] = s0;
        if (MODE == 1) { cx[r][iz] = s1; cy[r][iz] = s2; }
      }
    }
  }

  // ---- z sweep: values at Gauss points, factors, transposed z contraction ----
  double s0[NR][NB], sx[NR][NB], sy[NR][NB];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int iz = 0; iz < NB; ++iz) { s0[r][iz] = 0.0; sx[r][iz] = 0.0; sy[r][iz] = 0.0; }

  const size_t tile_qp = (size_t)QT * QT * QT;
  const double* ftile = fac + (size_t)tile * tile_qp * (MODE == 1 ? 6 : 1);
#pragma unroll
  for (int ez = 0; ez < TE; ++ez) {
#pragma unroll
    for (int jz = 0; jz < Q; ++jz) {
      const int qz = ez * Q + jz;
      const double* bz = &sB[2][(ez * Q + jz) * (P + 1)];
      if (MODE == 1) {
        const double* dz = &sD[2][(ez * Q + jz) * (P + 1)];
        const double* gq = ftile + (size_t)qz * 6 * QT * QT + tid;
        const double gxx = gq[0], gxy = gq[NT], gxz = gq[2 * NT];
        const double gyy = gq[3 * NT], gyz = gq[4 * NT], gzz = gq[5 * NT];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          double ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
          for (int c = 0; c <= P; ++c) {
            ux += bz[c] * cx[r][ez + c];
            uy += bz[c] * cy[r][ez + c];
            uz += dz[c] * c0[r][ez + c];
          }
          const double fx = gxx * ux + gxy * uy + gxz * uz;
          const double fy = gxy * ux + gyy * uy + gyz * uz;
          const double fz = gxz * ux + gyz * uy + gzz * uz;
#pragma unroll
          for (int c = 0; c <= P; ++c) {
            sx[r][ez + c] += bz[c] * fx;
            sy[r][ez + c] += bz[c] * fy;
            s0[r][ez + c] += dz[c] * fz;
          }
        }
      } else {
        const double wq = ftile[(size_t)qz * NT + tid];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          double u = 1.0;
          if (MODE == 0) {
            u = 0.0;
#pragma unroll
            for (int c = 0; c <= P; ++c) u += bz[c] * c0[r][ez + c];
          }
          const double v = wq * u;
#pragma unroll
          for (int c = 0; c <= P; ++c) s0[r][ez + c] += bz[c] * v;
        }
      }
    }
  }

  // ---- transposed y and x contractions, one coefficient plane at a time ----
  const int ncomp = NG;
#pragma unroll
  for (int iz = 0; iz < NB; ++iz) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double* S = &work[r][0];
      if (MODE == 1) {
        S[tid] = sx[r][iz];
        S[NT + tid] = sy[r][iz];
        S[2 * NT + tid] = s0[r][iz];
      } else {
        S[tid] = s0[r][iz];
      }
    }
    __syncthreads();
    // R[c][iy][qx]: c = 0 pairs with Dx (stiffness) or Bx (mass); c = 1 pairs with Bx
    constexpr int NRV = (MODE == 1 ? 2 : 1) * NB * QT;
    for (int i = tid; i < NR * NRV; i += NT) {
      int r = i / NRV, b = i % NRV;
      int q = b % QT, iy = (b / QT) % NB, c = b / (NB * QT);
      const double* S = &work[r][0];
      double acc = 0.0;
#pragma unroll
      for (int ey = 0; ey < TE; ++ey) {
        int a = iy - ey;
        if (a < 0 || a > P) continue;
#pragma unroll
        for (int jy = 0; jy < Q; ++jy) {
          int qyy = ey * Q + jy;
          double bvy = sB[1][(ey * Q + jy) * (P + 1) + a];
          if (MODE == 1) {
            if (c == 0) {
              acc += bvy * S[qyy * QT + q];
            } else {
              double dvy = sD[1][(ey * Q + jy) * (P + 1) + a];
              acc += dvy * S[NT + qyy * QT + q] + bvy * S[2 * NT + qyy * QT + q];
            }
          } else {
            acc += bvy * S[qyy * QT + q];
          }
        }
      }
      work[r][ncomp * NT + b] = acc;
    }
    __syncthreads();
    for (int i = tid; i < NR * NPL; i += NT) {
      int r = i / NPL, b = i % NPL;
      int ix = b % NB, iy = b / NB;
      const double* R = &work[r][ncomp * NT];
      double acc = 0.0;
#pragma unroll
      for (int ex = 0; ex < TE; ++ex) {
        int a = ix - ex;
        if (a < 0 || a > P) continue;
#pragma unroll
        for (int jx = 0; jx < Q; ++jx) {
          int q = ex * Q + jx;
          if (MODE == 1)
            acc += sD[0][(ex * Q + jx) * (P + 1) + a] * R[iy * QT + q] +
                   sB[0][(ex * Q + jx) * (P + 1) + a] * R[NB * QT + iy * QT + q];
          else
            acc += sB[0][(ex * Q + jx) * (P + 1) + a] * R[iy * QT + q];
        }
      }
      long long f = free_index3(g, e0[0] + ix, e0[1] + iy, e0[2] + iz);
      if (f >= 0) unsafeAtomicAdd(&y[(size_t)r * n_free + f], alpha * acc);
    }
  }
}

// Geometry factors at the Gauss points of one tile (setup, once per patch).
template <int P>
__global__ void __launch_bounds__(Tile3<P>::NT)
geo3d_kernel(const double* __restrict__ ctrl,  // [3][N_dof] full grid, co-lex
             const double* __restrict__ tB0, const double* __restrict__ tB1,
             const double* __restrict__ tB2, const double* __restrict__ tD0,
             const double* __restrict__ tD1, const double* __restrict__ tD2,
             const double* __restrict__ w0, const double* __restrict__ w1,
             const double* __restrict__ w2, Geo3 g, double* __restrict__ W,
             double* __restrict__ G, int* __restrict__ bad) {
  using T = Tile3<P>;
  constexpr int Q = T::Q, QT = T::QT, NT = T::NT, TE = T::TE;
  const int tid = threadIdx.x;
  const int qx = tid % QT, qy = tid / QT;
  const long long tile = blockIdx.x;
  const int tx = (int)(tile % g.nt[0]);
  const int ty = (int)((tile / g.nt[0]) % g.nt[1]);
  const int tz = (int)(tile / ((long long)g.nt[0] * g.nt[1]));
  const int ex = tx * TE + qx / Q, jx = qx % Q;
  const int ey = ty * TE + qy / Q, jy = qy % Q;
  const long long ndof = (long long)g.m[0] * g.m[1] * g.m[2];
  const size_t tile_qp = (size_t)QT * QT * QT;
  for (int qz = 0; qz < QT; ++qz) {
    const int ez = tz * TE + qz / Q, jz = qz % Q;
    const size_t wi = (size_t)tile * tile_qp + (size_t)qz * NT + tid;
    const size_t gi = (size_t)tile * tile_qp * 6 + (size_t)qz * 6 * NT + tid;
    if (ex >= g.n[0] || ey >= g.n[1] || ez >= g.n[2]) {
      W[wi] = 0.0;
      for (int c = 0; c < 6; ++c) G[gi + (size_t)c * NT] = 0.0;
      continue;
    }
    const double* bx = &tB0[((size_t)ex * Q + jx) * (P + 1)];
    const double* dx = &tD0[((size_t)ex * Q + jx) * (P + 1)];
    const double* by = &tB1[((size_t)ey * Q + jy) * (P + 1)];
    const double* dy = &tD1[((size_t)ey * Q + jy) * (P + 1)];
    const double* bz = &tB2[((size_t)ez * Q + jz) * (P + 1)];
    const double* dz = &tD2[((size_t)ez * Q + jz) * (P + 1)];
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int c2 = 0; c2 <= P; ++c2)
      for (int c1 = 0; c1 <= P; ++c1)
        for (int c0 = 0; c0 <= P; ++c0) {
          long long idx = (ex + c0) + (long long)g.m[0] * ((ey + c1) + (long long)g.m[1] * (ez + c2));
          double d0 = dx[c0] * by[c1] * bz[c2];
          double d1 = bx[c0] * dy[c1] * bz[c2];
          double d2 = bx[c0] * by[c1] * dz[c2];
          for (int c = 0; c < 3; ++c) {
            double cp = ctrl[(size_t)c * ndof + idx];
            J[c][0] += cp * d0;
            J[c][1] += cp * d1;
            J[c][2] += cp * d2;
          }
        }
    // adjugate: J^{-1} = adj / det
    double A[3][3];
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
    if (!(det > 0.0)) atomicOr(bad, 1);
    const double wq = w0[(size_t)ex * Q + jx] * w1[(size_t)ey * Q + jy] * w2[(size_t)ez * Q + jz];
    const double wdet = wq * det;
    W[wi] = wdet;
    // G = w det J^{-1} J^{-T} = (w / det) adj adj^T
    const double sc = wq / det;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      for (int t = 0; t < 3; ++t) v += A[ia[c]][t] * A[ib[c]][t];
      G[gi + (size_t)c * NT] = sc * v;
    }
  }
}

template <int P>
static int launch_op3d_p(int mode, int nr, const ga_patch* pt, const double* x, double* y,
                         double alpha, hipStream_t st) {
  using T = Tile3<P>;
  Geo3 g;
  for (int a = 0; a < 3; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.nt[a] = pt->nt[a]; }
  dim3 grid((unsigned)pt->n_tiles), block(T::NT);
  const double* const* B = (mode == 2) ? pt->tabB2 : pt->tabB;
  const double* fac = (mode == 1) ? pt->G : pt->W;
#define GA_OP3(MODE, NRV)                                                                   \
  hipLaunchKernelGGL((op3d_kernel<P, MODE, NRV>), grid, block, 0, st, x, y, fac, B[0], B[1], \
                     B[2], pt->tabD[0], pt->tabD[1], pt->tabD[2], g, pt->n_free, alpha)
  if (mode == 0) {
    if (nr == 1) GA_OP3(0, 1); else if (nr == 2) GA_OP3(0, 2); else GA_OP3(0, 3);
  } else if (mode == 1) {
    if (nr == 1) GA_OP3(1, 1); else if (nr == 2) GA_OP3(1, 2); else GA_OP3(1, 3);
  } else {
    GA_OP3(2, 1);
  }
#undef GA_OP3
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_op3d(int mode, int nr, const ga_patch* pt, const double* x, double* y, double alpha,
                hipStream_t st) {
  switch (pt->p) {
    case 1: return launch_op3d_p<1>(mode, nr, pt, x, y, alpha, st);
    case 2: return launch_op3d_p<2>(mode, nr, pt, x, y, alpha, st);
    case 3: return launch_op3d_p<3>(mode, nr, pt, x, y, alpha, st);
    case 4: return launch_op3d_p<4>(mode, nr, pt, x, y, alpha, st);
  }
  return -1;
}

int launch_geo3d(const ga_patch* pt, const double* ctrl, const double* const* w, int* bad,
                 hipStream_t st) {
  Geo3 g;
  for (int a = 0; a < 3; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.nt[a] = pt->nt[a]; }
#define GA_GEO3(PP)                                                                           \
  hipLaunchKernelGGL(geo3d_kernel<PP>, dim3((unsigned)pt->n_tiles), dim3(Tile3<PP>::NT), 0, st, \
                     ctrl, pt->tabB[0], pt->tabB[1], pt->tabB[2], pt->tabD[0], pt->tabD[1],    \
                     pt->tabD[2], w[0], w[1], w[2], g, pt->W, pt->G, bad)
  switch (pt->p) {
    case 1: GA_GEO3(1); break;
    case 2: GA_GEO3(2); break;
    case 3: GA_GEO3(3); break;
    case 4: GA_GEO3(4); break;
    default: return -1;
  }
#undef GA_GEO3
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int tile_threads3(int p) { return (TE3 * (p + 1)) * (TE3 * (p + 1)); }

}  // namespace ga
