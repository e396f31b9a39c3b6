// 3-D operator launches in FP64, the geometry-factor kernel and the multi-patch
// tile-queue launches; the kernel templates are in ops3d_body.h.
#include "ops3d_body.h"

namespace ga {

// Geometry factors at the Gauss points of one element layer of one
// stiffness-layout xy tile; W is written in the mass-kernel tiling.
template <int P>
__global__ void __launch_bounds__((Tile3<P, te3_stiff(P)>::NT))
geo3d_kernel(const double* __restrict__ ctrl,  // [3][N_dof] full grid, co-lex
             const double* __restrict__ tB0, const double* __restrict__ tB1,
             const double* __restrict__ tB2, const double* __restrict__ tD0,
             const double* __restrict__ tD1, const double* __restrict__ tD2,
             const double* __restrict__ w0, const double* __restrict__ w1,
             const double* __restrict__ w2, Geo3 gk, int ntm0, double* __restrict__ W,
             double* __restrict__ G, int* __restrict__ bad) {
  using T = Tile3<P, te3_stiff(P)>;
  using TM = Tile3<P, te3_mass(P)>;
  constexpr int Q = T::Q, QT = T::QT, NT = T::NT, TE = T::TE;
  const int tid = threadIdx.x;
  const int qx = tid % QT, qy = tid / QT;
  const int txy = blockIdx.x, ez = blockIdx.y;
  const int tx = txy % gk.nt[0], ty = txy / gk.nt[0];
  const int ex = tx * TE + qx / Q, jx = qx % Q;
  const int ey = ty * TE + qy / Q, jy = qy % Q;
  if (ex >= gk.n[0] || ey >= gk.n[1]) return;  // padding: W and G stay zero
  const long long ndof = (long long)gk.m[0] * gk.m[1] * gk.m[2];
  const int qz_tot = gk.n[2] * Q;
  // global Gauss indices in x, y and the mass-layout position
  const int gx = tx * QT + qx, gy = ty * QT + qy;
  const int tm = gx / TM::QT + ntm0 * (gy / TM::QT);
  const int lm = (gy % TM::QT) * TM::QT + gx % TM::QT;
  for (int jz = 0; jz < Q; ++jz) {
    const int qz = ez * Q + jz;
    const size_t wi = ((size_t)tm * qz_tot + qz) * TM::NT + lm;
    const size_t gi = ((size_t)txy * qz_tot + qz) * 6 * NT + 2 * (size_t)tid;
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
          long long idx = (ex + c0) + (long long)gk.m[0] * ((ey + c1) + (long long)gk.m[1] * (ez + c2));
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
    W[wi] = wq * det;
    // G = w det J^{-1} J^{-T} = (w / det) adj adj^T
    const double sc = wq / det;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int c = 0; c < 6; ++c) {
      double v = 0.0;
      for (int t = 0; t < 3; ++t) v += A[ia[c]][t] * A[ib[c]][t];
      G[gi + (size_t)(c / 2) * 2 * NT + (c % 2)] = sc * v;   // components in pairs per thread
    }
  }
}

// element layers per workgroup: enough workgroups to fill the chip several times
int launch_op3d(int mode, int nr, const ga_patch* pt, const double* x, double* y, double alpha,
                hipStream_t st, const double* gate) {
  const double* fac = (mode == 1) ? pt->G : pt->W;
  switch (pt->p) {
    case 1: return launch_op3d_p<1, double>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 2: return launch_op3d_p<2, double>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 3: return launch_op3d_p<3, double>(mode, nr, pt, x, y, alpha, fac, st, gate);
    case 4: return launch_op3d_p<4, double>(mode, nr, pt, x, y, alpha, fac, st, gate);
  }
  return -1;
}


// tiles of one patch in the layout of `mode` with ze element layers per tile
long long op3d_tiles(int mode, const ga_patch* pt, int ze) {
  const int* nt = mode == 1 ? pt->ntk : pt->ntm;
  return (long long)nt[0] * nt[1] * ((pt->n[2] + ze - 1) / ze);
}

int op3d_default_ze(int mode, const ga_patch* pt, bool f32) {
  const int* nt = mode == 1 ? pt->ntk : pt->ntm;
  if (pt->ze > 0) return pt->ze;
  // tuned counts hold for the FP64 launches they were measured on
  if (!f32 && mode <= 1 && pt->ze_op[mode] > 0) return pt->ze_op[mode];
  return pick_ze((long long)nt[0] * nt[1], pt->n[2], mode == 1 ? 8 : 16);
}

OpGroupEntry op3d_group_entry(int mode, const ga_patch* pt, int ze, long long off, int tile0,
                              bool f32) {
  OpGroupEntry d;
  for (int a = 0; a < 3; ++a) {
    d.g.n[a] = pt->n[a]; d.g.m[a] = pt->m[a]; d.g.mf[a] = pt->mf[a]; d.g.lo[a] = pt->lo[a];
    d.tB[a] = pt->tabB[a];
    d.tD[a] = pt->tabD[a];
  }
  const int* nt = mode == 1 ? pt->ntk : pt->ntm;
  d.g.nt[0] = nt[0];
  d.g.nt[1] = nt[1];
  d.fac = mode == 1 ? (const void*)pt->G : (f32 ? (const void*)pt->W32 : (const void*)pt->W);
  d.ze = ze;
  d.off = off;
  d.tile0 = tile0;
  d.ntiles = (int)op3d_tiles(mode, pt, ze);
  d.sys = 0;
  return d;
}

template <int P, typename S>
static int group_p(int mode, int nr, const OpGroupEntry* ents, int nent, const S* x, S* y,
                   long long stride, S alpha, int total, int nwg, hipStream_t st, BatchGate gate) {
  constexpr int TK = te3_stiff(P), TM = te3_mass(P);
  const int per = (total + nwg - 1) / nwg;
  const dim3 grid((unsigned)((total + per - 1) / per));
#define GA_OPG(TE, MODE, NRV)                                                                    \
  hipLaunchKernelGGL((op3d_group_kernel<P, TE, MODE, NRV, S>), grid, dim3(Tile3<P, TE>::NT), 0, st, \
                     ents, nent, x, y, stride, alpha, total, per, gate)
  if (mode == 0) {
    if (nr == 1) GA_OPG(TM, 0, 1); else if (nr == 2) GA_OPG(TM, 0, 2); else GA_OPG(TM, 0, 3);
  } else {
    if constexpr (sizeof(S) == 8) {
      if (nr == 1) GA_OPG(TK, 1, 1); else if (nr == 2) GA_OPG(TK, 1, 2); else GA_OPG(TK, 1, 3);
    } else {
      return -1;
    }
  }
#undef GA_OPG
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename S>
int launch_op3d_group(int p, int mode, int nr, const OpGroupEntry* ents, int nent, const S* x,
                      S* y, long long stride, S alpha, int total, int nwg, hipStream_t st,
                      BatchGate gate) {
  if (nr < 1 || nr > 3 || total < 1 || nwg < 1 || (mode != 0 && mode != 1)) return -1;
  switch (p) {
    case 2: return group_p<2, S>(mode, nr, ents, nent, x, y, stride, alpha, total, nwg, st, gate);
    case 3: return group_p<3, S>(mode, nr, ents, nent, x, y, stride, alpha, total, nwg, st, gate);
    case 4: return group_p<4, S>(mode, nr, ents, nent, x, y, stride, alpha, total, nwg, st, gate);
  }
  return -1;
}
template int launch_op3d_group<double>(int, int, int, const OpGroupEntry*, int, const double*,
                                       double*, long long, double, int, int, hipStream_t,
                                       BatchGate);
template int launch_op3d_group<float>(int, int, int, const OpGroupEntry*, int, const float*,
                                      float*, long long, float, int, int, hipStream_t, BatchGate);

int launch_geo3d(const ga_patch* pt, const double* ctrl, const double* const* w, int* bad,
                 hipStream_t st) {
  Geo3 g;
  for (int a = 0; a < 3; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.lo[a] = pt->lo[a]; }
  g.nt[0] = pt->ntk[0];
  g.nt[1] = pt->ntk[1];
  dim3 grid((unsigned)(pt->ntk[0] * pt->ntk[1]), (unsigned)pt->n[2]);
#define GA_GEO3(PP)                                                                           \
  hipLaunchKernelGGL(geo3d_kernel<PP>, grid, dim3(Tile3<PP, te3_stiff(PP)>::NT), 0, st, ctrl,  \
                     pt->tabB[0], pt->tabB[1], pt->tabB[2], pt->tabD[0], pt->tabD[1],          \
                     pt->tabD[2], w[0], w[1], w[2], g, pt->ntm[0], pt->W, pt->G, bad)
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

}  // namespace ga
