// Sum-factorised 3-D operator kernels (shared by the FP64 and the low-precision
// translation units).
//
// 3-D sum-factorised operator kernels for gfx950.
//
//   y += alpha * B^T diag(W) B x                        (mass, eq. mass_matrix)
//   y += alpha * sum_ab D_a^T diag(G_ab) D_b x           (stiffness, K of eq. mp)
//   y += (B o B)^T W                                     (diag(M), the D of Sec. 5.4)
//
// with B = Bz (x) By (x) Bx the tensor basis at the Gauss points and
// W = w|det J|, G = w|det J| J^{-1} J^{-T} stored per Gauss point.
//
// Design (z-marching): one workgroup owns an xy column of TE x TE elements
// and a range of element layers along z.  Its (TE*Q)^2 threads each own one
// (qx, qy) line of Gauss points (Q = p+1 per element).  The workgroup marches
// up its z range one Gauss layer at a time and keeps the p+1 coefficient
// planes the current element layer touches in registers:
//   forward   a new coefficient plane (prefetched one element layer ahead)
//             is staged in LDS, contracted along x (LDS) and along y
//             (registers) into c[f][p] for the fields f needed at the Gauss
//             points (value; or x-, y-derivatives and value);
//   z sweep   per Gauss layer: contraction along z, the 1 or 6 quadrature
//             factors (a small ring prefetches the next layers; the factor
//             stream is contiguous along z, read once with nontemporal, fully
//             coalesced loads) and the transposed z contraction into
//             accumulators s[f][p];
//   backward  the plane no later layer touches is finished: transposed y and
//             x contractions with zero-padded transposed basis tables in LDS
//             (dense products for the mass; for the stiffness only the taps of
//             the elements each basis function touches), then FP64 atomic adds
//             into y (xy neighbours and the two ends of a z range share planes).
// The stiffness kernel uses 4x4-element columns (6 factors per point, high
// register use); the mass kernels use wider columns so the fixed per-plane
// work is spread over more Gauss points.
// Factor layout: W [xy tile][qz over the whole z extent][qy][qx]; G [xy tile]
// [qz][component pair][qy][qx][2] (each thread reads its 6 components as three
// 16-byte pairs).
#pragma once
#include <hip/hip_runtime.h>

#include "ga_internal.h"
#include "kernels.h"

namespace ga {

template <int P, int TE_>
struct Tile3 {
  static constexpr int Q = P + 1;
  static constexpr int TE = TE_;
  static constexpr int QT = TE * Q;      // Gauss points per tile edge
  static constexpr int NB = TE + P;      // coefficients per tile edge
  static constexpr int NT = QT * QT;     // threads per workgroup
  static constexpr int TAB = TE * Q * (P + 1);
};


// index of a full-grid coefficient (i0,i1,i2) in the free vector, or -1
inline __device__ __forceinline__ long long free_index3(const Geo3& g, int i0, int i1, int i2) {
  int f0 = i0 - g.lo[0], f1 = i1 - g.lo[1], f2 = i2 - g.lo[2];
  if (f0 < 0 || f1 < 0 || f2 < 0 || f0 >= g.mf[0] || f1 >= g.mf[1] || f2 >= g.mf[2]) return -1;
  return (long long)f0 + (long long)g.mf[0] * (f1 + (long long)g.mf[1] * f2);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tiles so xy/z neighbours share its L2.
inline __device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned nwg) {
  const unsigned nx = 8;
  const unsigned per = nwg / nx, rem = nwg % nx;
  const unsigned xcd = bid % nx, loc = bid / nx;
  const unsigned base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
  return base + loc;
}

#ifndef GA_OP3_WAVES_K
#define GA_OP3_WAVES_K 2
#endif
#ifndef GA_OP3_WAVES_M
#define GA_OP3_WAVES_M 1
#endif
// Gauss layers of quadrature factors prefetched ahead (stiffness: 6 factors per
// point and much arithmetic per layer; mass: 1 factor and little arithmetic, so a
// deeper ring is needed to cover the memory latency)
#ifndef GA_RING_K
#define GA_RING_K 4
#endif
// p = 4 stiffness with two right-hand sides: a ring of 2 keeps the field
// planes within the register budget of two waves per SIMD
constexpr int stiff_ring(int P, int NR) { return (P == 4 && NR >= 2) ? 2 : GA_RING_K; }
// mass ring by degree and right-hand-side count (measured at 128^3 p = 2, 3 and
// 96^3 p = 4); GA_RING_M overrides it for every case
constexpr int mass_ring(int P, int NR) {
#ifdef GA_RING_M
  return GA_RING_M;
#else
  return P == 3 ? 16 : (P == 2 ? (NR == 1 ? 4 : 16) : (NR == 1 ? 16 : 4));
#endif
}

// Value held by lane (l ^ 1) of the wave (DPP quad permutation [1,0,3,2]); both
// lanes of the pair must be active.
inline __device__ __forceinline__ double lane_xor1(double v) {
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
inline __device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// MODE: 0 mass, 1 stiffness, 2 diag(M) (tables hold squared values, x unused)
// One workgroup's share: logical tile `lid` = (xy column, z range) of one patch.
// x and y hold NR right-hand sides `n_free` entries apart.
// BW selects the backward stages: 0 dense products (any MODE), 1 dense y stage and
// the x stage with two lanes per coefficient (mass), 2 both stages over the
// supporting elements only (stiffness).  F is the storage type of the quadrature
// factors: S itself, or BF16 (F = unsigned short, bit patterns) widened to S.
template <int P, int TE, int MODE, int NR, typename S, int BW, typename F>
__device__ __forceinline__ void
op3d_body(const S* __restrict__ x, S* __restrict__ y,
          const F* __restrict__ fac,
          const double* __restrict__ tB0, const double* __restrict__ tB1,
          const double* __restrict__ tB2, const double* __restrict__ tD0,
          const double* __restrict__ tD1, const double* __restrict__ tD2,
          Geo3 g, int ze, long long n_free, S alpha, unsigned lid) {
  using T = Tile3<P, TE>;
  constexpr int Q = T::Q, QT = T::QT, NB = T::NB, NT = T::NT;
  constexpr int NPL = NB * NB;                  // coefficients per plane of the box
  constexpr int NF = (MODE == 1) ? 3 : 1;       // fields at the Gauss points
  constexpr int NA = (MODE == 1) ? 2 : 1;       // x-contracted fields
  constexpr int NFY = (BW == 2) ? 3 : (MODE == 1 ? 2 : 1);  // y-back-contracted rows per RHS
  constexpr int NC = (MODE == 1) ? 6 : 1;       // factor components per Gauss point
  constexpr int XPR = (NR * NPL + NT - 1) / NT; // prefetched plane values per thread
  constexpr int QP = QT + 1;                    // padded LDS row (no bank conflicts)

  __shared__ S sB[2][T::TAB];
  __shared__ S sD[2][T::TAB];
  // x tables by local index: xB[a][q] = value of basis ex(q)+a at tile Gauss point q
  __shared__ S xB[P + 1][QT];
  __shared__ S xD[P + 1][QT];
  // transposed, zero-padded: tBs[a][i * QP + q] = basis i of the box at tile Gauss point q
  __shared__ S tBs[2][NB * QP];
  __shared__ S tDs[2][NB * QP];
  __shared__ S Xs[NR][NPL];
  __shared__ S As[NR][NA][NB * QT];
  __shared__ S Ss[NR][NF][NT];
  __shared__ S Rs[NR][NFY][NB * QP];
  // box indices 0..NB-1 ordered by decreasing number of elements of the tile their
  // basis function touches (the middle ones first): the stiffness's y-stage rows in
  // this order have nearly equal trip counts within a wave
  __shared__ int ordv[NB];

  const int tid = threadIdx.x;
  const int qx = tid % QT, qy = tid / QT;
  const int ntxy = g.nt[0] * g.nt[1];
  const int txy = (int)(lid % ntxy);
  const int zc = (int)(lid / ntxy);
  const int tx = txy % g.nt[0], ty = txy / g.nt[0];
  const int e0x = tx * TE, e0y = ty * TE;
  const int ez0 = zc * ze;
  const int ez1 = min(ez0 + ze, g.n[2]);
  const int qz_tot = g.n[2] * Q;

  for (int i = tid; i < T::TAB; i += NT) {
    sB[0][i] = (S)tB0[(size_t)e0x * Q * (P + 1) + i];
    sB[1][i] = (S)tB1[(size_t)e0y * Q * (P + 1) + i];
    if (MODE == 1) {
      sD[0][i] = (S)tD0[(size_t)e0x * Q * (P + 1) + i];
      sD[1][i] = (S)tD1[(size_t)e0y * Q * (P + 1) + i];
    }
  }
  for (int i = tid; i < 2 * NB * QT; i += NT) {
    const int ax = i / (NB * QT), b = i % (NB * QT);
    const int ib = b / QT, q = b % QT;
    const int el = q / Q, jq = q % Q, a = ib - el;
    const double* tb = ax == 0 ? tB0 + (size_t)e0x * Q * (P + 1) : tB1 + (size_t)e0y * Q * (P + 1);
    const double* td = ax == 0 ? tD0 + (size_t)e0x * Q * (P + 1) : tD1 + (size_t)e0y * Q * (P + 1);
    const bool in = a >= 0 && a <= P;
    tBs[ax][ib * QP + q] = in ? (S)tb[(el * Q + jq) * (P + 1) + a] : (S)0;
    tDs[ax][ib * QP + q] = (in && MODE == 1) ? (S)td[(el * Q + jq) * (P + 1) + a] : (S)0;
  }
  for (int i = tid; i < (P + 1) * QT; i += NT) {
    const int a = i / QT, q = i % QT;
    xB[a][q] = (S)tB0[(size_t)e0x * Q * (P + 1) + q * (P + 1) + a];
    xD[a][q] = MODE == 1 ? (S)tD0[(size_t)e0x * Q * (P + 1) + q * (P + 1) + a] : (S)0;
  }
  if (BW == 2 && tid == 0) {
    int j = 0;
    for (int ne = (P + 1 < TE ? P + 1 : TE); ne >= 1; --ne)
      for (int i = 0; i < NB; ++i)
        if (min(TE - 1, i) - max(0, i - P) + 1 == ne) ordv[j++] = i;
  }
  const int eyq = qy / Q, jyq = qy % Q;
  const F* fcol = fac + (size_t)txy * qz_tot * NC * NT + tid;
  // factors of Gauss layer q: the stiffness stores its 6 components as 3 pairs
  // per thread ([layer][pair][thread][2]), read with 16-byte loads
  // The factor stream is read exactly once per apply: nontemporal loads keep it from
  // displacing the coefficient vectors (re-read by neighbouring tiles) in the caches.
  auto load_fac = [&](int q, S (&dst)[NC]) {
    if constexpr (sizeof(F) == 2) {
      // BF16: a component pair is one 32-bit word (first component in the low half)
      if constexpr (MODE == 1) {
        const unsigned* b2 =
            reinterpret_cast<const unsigned*>(fac + ((size_t)txy * qz_tot + q) * NC * NT) + tid;
#pragma unroll
        for (int h = 0; h < NC / 2; ++h) {
          const unsigned v = __builtin_nontemporal_load(b2 + (size_t)h * NT);
          dst[2 * h] = (S)__uint_as_float(v << 16);
          dst[2 * h + 1] = (S)__uint_as_float(v & 0xffff0000u);
        }
      } else {
        const unsigned short v = __builtin_nontemporal_load(fcol + (size_t)q * NT);
        dst[0] = (S)__uint_as_float((unsigned)v << 16);
      }
    } else if constexpr (MODE == 1) {
      typedef S V2 __attribute__((ext_vector_type(2)));
      const V2* b2 = reinterpret_cast<const V2*>(fac + ((size_t)txy * qz_tot + q) * NC * NT) + tid;
#pragma unroll
      for (int h = 0; h < NC / 2; ++h) {
        const V2 v = __builtin_nontemporal_load(b2 + (size_t)h * NT);
        dst[2 * h] = v.x;
        dst[2 * h + 1] = v.y;
      }
    } else {
      dst[0] = __builtin_nontemporal_load(fcol + (size_t)q * NT);
    }
  };

  S c[NR][NF][P + 1];   // forward fields of the coefficient planes ez..ez+P
  S s[NR][NF][P + 1];   // transposed-z accumulators of the same planes
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int j = 0; j <= P; ++j) { c[r][f][j] = 0.0; s[r][f][j] = 0.0; }

  // prefetch of the next coefficient plane (global -> registers)
  S xpre[XPR];
  auto load_plane = [&](int iz) {
#pragma unroll
    for (int k = 0; k < XPR; ++k) {
      const int i = tid + k * NT;
      S v = 0.0;
      if (i < NR * NPL) {
        const int r = i / NPL, b = i % NPL;
        const long long f = free_index3(g, e0x + b % NB, e0y + b / NB, iz);
        if (f >= 0) v = x[(size_t)r * n_free + f];
      }
      xpre[k] = v;
    }
  };

  // backward, y stage: Rs[r][f][iy][q] = sum over the Gauss rows k of the elements
  // that basis iy touches of W_f(iy, k) Ss[r][f][k][q], W = y derivative (field 1 of
  // the stiffness) or value.  Stiffness: one field per row, rows in ordv order, q
  // fastest, only the nonzero taps (half the work of the dense product and no mixed
  // one- and two-field items within a wave)
  auto back_y = [&]() {
    if constexpr (BW != 2) {
      // dense products with the zero-padded transposed table over all Gauss rows of
      // the tile; the stiffness sums its fields 1 and 2 in one row
      int lz = 0;
      asm volatile("" : "+v"(lz));
      for (int i = tid; i < NR * NFY * NB * QT; i += NT) {
        const int r = i / (NFY * NB * QT), b = i % (NFY * NB * QT);
        const int q = b % QT, iy = (b / QT) % NB, cf = b / (NB * QT);
        const S* ty_ = &tBs[1][iy * QP + lz];
        const S* tdy = &tDs[1][iy * QP + lz];
        S acc = 0.0;
        if (MODE == 1 && cf == 1) {
#pragma unroll 4
          for (int k = 0; k < QT; ++k)
            acc += tdy[k] * Ss[r][1][k * QT + q] + ty_[k] * Ss[r][2][k * QT + q];
        } else {
#pragma unroll 4
          for (int k = 0; k < QT; ++k) acc += ty_[k] * Ss[r][0][k * QT + q];
        }
        Rs[r][cf][iy * QP + q] = acc;
      }
      return;
    }
    for (int i = tid; i < NB * NR * NFY * QT; i += NT) {
      const int q = i % QT, row = i / QT;
      const int f = row % NFY, r = (row / NFY) % NR, iy = ordv[row / (NFY * NR)];
      const S* w = (MODE == 1 && f == 1) ? &tDs[1][iy * QP] : &tBs[1][iy * QP];
      const S* src = &Ss[r][f][q];
      const int k1 = (min(TE - 1, iy) + 1) * Q;
      S acc = 0.0;
      for (int k = max(0, iy - P) * Q; k < k1; k += Q) {
#pragma unroll
        for (int j = 0; j < Q; ++j) acc += w[k + j] * src[(k + j) * QT];
      }
      Rs[r][f][iy * QP + q] = acc;
    }
  };
  // backward, x stage and the atomic adds of plane iz: coefficient (ix, iy) sums
  // over the Gauss points of the elements basis ix touches (x derivative for field
  // 0 of the stiffness, value otherwise).  BW 1, 2: two lanes share a coefficient,
  // each taking every other element, combined by a lane exchange (every thread runs
  // the same number of rounds); coefficients in x-fastest order, so the atomic adds
  // of a wave fall on few cache lines (half the write traffic of the support order).
  // BW 0: one lane per coefficient, dense product.
  auto back_x = [&](int iz) {
    if constexpr (BW == 0) {
      int lz = 0;
      asm volatile("" : "+v"(lz));
      for (int i = tid; i < NR * NPL; i += NT) {
        const int r = i / NPL, b = i % NPL;
        const int ix = b % NB, iy = b / NB;
        const S* tx_ = &tBs[0][ix * QP + lz];
        const S* tdx = &tDs[0][ix * QP + lz];
        S acc = 0.0;
#pragma unroll 4
        for (int k = 0; k < QT; ++k) {
          if (MODE == 1) acc += tdx[k] * Rs[r][0][iy * QP + k] + tx_[k] * Rs[r][1][iy * QP + k];
          else acc += tx_[k] * Rs[r][0][iy * QP + k];
        }
        const long long f = free_index3(g, e0x + ix, e0y + iy, iz);
        if (f >= 0) unsafeAtomicAdd(&y[(size_t)r * n_free + f], alpha * acc);
      }
      return;
    }
    constexpr int NX = 2 * NB * NR * NB;
    // the pair (l, l ^ 1) must be the lane pair (tid, tid ^ 1) of one wave: true when
    // every round starts at an even l (even NT) or there is a single round
    static_assert(BW == 0 || NT % 2 == 0 || NX <= NT, "two-lane x stage needs aligned lane pairs");
    for (int i0 = 0; i0 < NX; i0 += NT) {
      const int l = i0 + tid, h = l & 1, it = l >> 1;
      const bool act = l < NX;
      const int ix = it % NB, iy = (it / NB) % NB, r = act ? it / NPL : 0;
      S acc = 0.0;
      if (act) {
        const int e1 = min(TE - 1, ix);
        for (int e = max(0, ix - P) + h; e <= e1; e += 2) {
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            const int k = e * Q + j;
            if constexpr (BW == 2)
              acc += tDs[0][ix * QP + k] * Rs[r][0][iy * QP + k] +
                     tBs[0][ix * QP + k] * (Rs[r][1][iy * QP + k] + Rs[r][NFY - 1][iy * QP + k]);
            else
              acc += tBs[0][ix * QP + k] * Rs[r][0][iy * QP + k];
          }
        }
      }
      acc += lane_xor1(acc);
      if (act && h == 0) {
        const long long f = free_index3(g, e0x + ix, e0y + iy, iz);
        if (f >= 0) unsafeAtomicAdd(&y[(size_t)r * n_free + f], alpha * acc);
      }
    }
  };

  // contract the prefetched plane along x (LDS) and y (registers) into c[.][.][P]
  auto forward_plane = [&]() {
    int lz = 0;
    asm volatile("" : "+v"(lz));  // keep the basis-table reads below in LDS (no hoisting)
#pragma unroll
    for (int k = 0; k < XPR; ++k) {
      const int i = tid + k * NT;
      if (i < NR * NPL) Xs[i / NPL][i % NPL] = xpre[k];
    }
    __syncthreads();
    for (int i = tid; i < NR * NB * QT; i += NT) {
      const int r = i / (NB * QT), b = i % (NB * QT);
      const int q = b % QT, iy = b / QT;
      const int ex = q / Q, jx = q % Q;
      const S* xs = &Xs[r][iy * NB + ex];
      S a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int a = 0; a <= P; ++a) a0 += xB[a][q + lz] * xs[a];
      As[r][0][b] = a0;
      if (MODE == 1) {
#pragma unroll
        for (int a = 0; a <= P; ++a) a1 += xD[a][q + lz] * xs[a];
        As[r][1][b] = a1;
      }
    }
    __syncthreads();
    const S* by = &sB[1][(eyq * Q + jyq) * (P + 1) + lz];
    const S* dy = &sD[1][(eyq * Q + jyq) * (P + 1) + lz];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      S v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
      for (int b = 0; b <= P; ++b) {
        const S a0 = As[r][0][(eyq + b) * QT + qx];
        v0 += by[b] * a0;
        if (MODE == 1) {
          v1 += by[b] * As[r][1][(eyq + b) * QT + qx];
          v2 += dy[b] * a0;
        }
      }
      if (MODE == 1) {
        c[r][0][P] = v1;  // d/dx (to be contracted with Bz)
        c[r][1][P] = v2;  // d/dy (Bz)
        c[r][2][P] = v0;  // value (Dz gives d/dz)
      } else {
        c[r][0][P] = v0;
      }
    }
  };

  // finish coefficient plane iz from s[.][.][0]: transposed y and x contractions
  auto backward_plane = [&](int iz) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f) Ss[r][f][tid] = s[r][f][0];
    __syncthreads();
    back_y();
    __syncthreads();
    back_x(iz);
  };

  auto shift_c_ = [&]() {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < P; ++j) c[r][f][j] = c[r][f][j + 1];
  };
  // finish plane iz (backward) and contract the prefetched plane (forward) in
  // one pass of two barriers: the two use disjoint LDS buffers
  auto step_planes = [&](int iz) {
    int lz = 0;
    asm volatile("" : "+v"(lz));
    // no barrier needed before these writes: Ss and Xs were last read before the
    // last barrier of the previous plane step (or forward/backward plane), and the
    // z sweep in between uses no LDS
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f) Ss[r][f][tid] = s[r][f][0];
#pragma unroll
    for (int k = 0; k < XPR; ++k) {
      const int i = tid + k * NT;
      if (i < NR * NPL) Xs[i / NPL][i % NPL] = xpre[k];
    }
    __syncthreads();
    back_y();
    for (int i = tid; i < NR * NB * QT; i += NT) {
      const int r = i / (NB * QT), b = i % (NB * QT);
      const int q = b % QT, iy = b / QT;
      const int ex = q / Q, jx = q % Q;
      const S* xs = &Xs[r][iy * NB + ex];
      S a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int a = 0; a <= P; ++a) a0 += xB[a][q + lz] * xs[a];
      As[r][0][b] = a0;
      if (MODE == 1) {
#pragma unroll
        for (int a = 0; a <= P; ++a) a1 += xD[a][q + lz] * xs[a];
        As[r][1][b] = a1;
      }
    }
    __syncthreads();
    back_x(iz);
    shift_c_();
    const S* by = &sB[1][(eyq * Q + jyq) * (P + 1) + lz];
    const S* dy = &sD[1][(eyq * Q + jyq) * (P + 1) + lz];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      S v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
      for (int b = 0; b <= P; ++b) {
        const S a0 = As[r][0][(eyq + b) * QT + qx];
        v0 += by[b] * a0;
        if (MODE == 1) {
          v1 += by[b] * As[r][1][(eyq + b) * QT + qx];
          v2 += dy[b] * a0;
        }
      }
      if (MODE == 1) {
        c[r][0][P] = v1;
        c[r][1][P] = v2;
        c[r][2][P] = v0;
      } else {
        c[r][0][P] = v0;
      }
    }
  };

  auto shift_c = [&]() {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int j = 0; j < P; ++j) c[r][f][j] = c[r][f][j + 1];
  };
  auto shift_s = [&]() {
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int j = 0; j < P; ++j) s[r][f][j] = s[r][f][j + 1];
        s[r][f][P] = 0.0;
      }
  };

  __syncthreads();
  if (MODE != 2) {
    load_plane(ez0);
#pragma unroll 1
    for (int j = 0; j <= P; ++j) {
      if (j > 0) shift_c();
      forward_plane();
      load_plane(ez0 + j + 1);   // plane ez0 + P + 1 is the first one of the march
    }
  }

  // z sweep over Gauss layers with a ring of D prefetched factor planes
  constexpr int D = (MODE == 1) ? stiff_ring(P, NR) : mass_ring(P, NR);
  const int q0 = ez0 * Q, q1 = ez1 * Q;
  S gq[D][NC];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (q0 + d < q1) {
      load_fac(q0 + d, gq[d]);
    } else {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) gq[d][cc] = 0.0;
    }
  }

  for (int qb = q0; qb < q1; qb += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int q = qb + d;
      if (q >= q1) break;
      const int ez = q / Q, jz = q - ez * Q;
      S cur[NC];
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) cur[cc] = gq[d][cc];
      if (q + D < q1) load_fac(q + D, gq[d]);
      const double* bzt = tB2 + ((size_t)ez * Q + jz) * (P + 1);
      const double* dzt = tD2 + ((size_t)ez * Q + jz) * (P + 1);
      S bz[P + 1], dz[P + 1];
#pragma unroll
      for (int a = 0; a <= P; ++a) {
        bz[a] = (S)bzt[a];
        if (MODE == 1) dz[a] = (S)dzt[a];
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (MODE == 1) {
          S ux = 0.0, uy = 0.0, uz = 0.0;
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            ux += bz[a] * c[r][0][a];
            uy += bz[a] * c[r][1][a];
            uz += dz[a] * c[r][2][a];
          }
          const S fx = cur[0] * ux + cur[1] * uy + cur[2] * uz;
          const S fy = cur[1] * ux + cur[3] * uy + cur[4] * uz;
          const S fz = cur[2] * ux + cur[4] * uy + cur[5] * uz;
#pragma unroll
          for (int a = 0; a <= P; ++a) {
            s[r][0][a] += bz[a] * fx;
            s[r][1][a] += bz[a] * fy;
            s[r][2][a] += dz[a] * fz;
          }
        } else {
          S u = 1.0;
          if (MODE == 0) {
            u = 0.0;
#pragma unroll
            for (int a = 0; a <= P; ++a) u += bz[a] * c[r][0][a];
          }
          const S v = cur[0] * u;
#pragma unroll
          for (int a = 0; a <= P; ++a) s[r][0][a] += bz[a] * v;
        }
      }
      if (jz == Q - 1) {
        // plane ez is complete; the next element layer needs plane ez + 1 + P
        if (MODE != 2 && ez + 1 < ez1) {
          step_planes(ez);  // backward of plane ez, forward of plane ez + 1 + P
          shift_s();
          if (ez + 2 < ez1) load_plane(ez + 2 + P);
        } else {
          backward_plane(ez);
          shift_s();
        }
      }
    }
  }
#pragma unroll 1
  for (int j = 0; j < P; ++j) {
    backward_plane(ez1 + j);
    shift_s();
  }
}

// Backward variant per instance (measured): the stiffness on up to two right-hand
// sides takes the support-limited stages; the single-patch p = 3 FP64 mass on one
// or two right-hand sides the two-lane x stage (its two-RHS instance then needs a
// bound of 4 waves per SIMD to keep its occupancy); every other instance the dense
// stages, where the extra registers would spill or cost occupancy.
template <int P, int MODE, int NR, typename S>
constexpr int op3d_backward() {
  return (MODE == 1 && NR <= 2) ? 2 : ((MODE == 0 && P == 3 && NR <= 2 && sizeof(S) == 8) ? 1 : 0);
}
template <int P, int MODE, int NR>
constexpr int op3d_group_backward() {
  return (MODE == 1 && NR <= 2 && P <= 3) ? 2 : 0;
}
template <int P, int MODE, int NR, typename S>
constexpr int op3d_waves() {
  return MODE == 1 ? GA_OP3_WAVES_K
                   : ((MODE == 0 && P == 3 && NR == 2 && sizeof(S) == 8) ? 4 : GA_OP3_WAVES_M);
}

// One colour class of tiles (deterministic mode): tiles (tx, ty, zc) with tx = a (mod
// cx), ty = b (mod cy), zc = c (mod cz), where the strides are large enough that two
// tiles of one class share no coefficient; the classes run one launch after the other,
// so every coefficient receives its contributions in a fixed order.  cx = 0: all tiles.
struct TileColor {
  int cx, cy, cz, a, b, c, nx, ny;  // nx, ny: tiles of the class along x and y
};

template <int P, int TE, int MODE, int NR, typename S, typename F = S>
__global__ void __launch_bounds__((Tile3<P, TE>::NT), (op3d_waves<P, MODE, NR, S>()))
op3d_kernel(const S* __restrict__ x, S* __restrict__ y,
            const F* __restrict__ fac,
            const double* __restrict__ tB0, const double* __restrict__ tB1,
            const double* __restrict__ tB2, const double* __restrict__ tD0,
            const double* __restrict__ tD1, const double* __restrict__ tD2,
            Geo3 g, int ze, long long n_free, S alpha, const double* __restrict__ gate,
            TileColor col) {
  // device-side control: with a gate (the CG scalars of the launch's first
  // right-hand side), the launch does nothing once all its systems have converged
  if (gate) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) any |= gate[r * NSCAL + S_ACTIVE] != 0.0;
    if (!any) return;
  }
  unsigned lid = xcd_remap(blockIdx.x, gridDim.x);
  if (col.cx) {
    const unsigned ix = lid % col.nx, iy = (lid / col.nx) % col.ny, iz = lid / (col.nx * col.ny);
    const unsigned tx = col.a + col.cx * ix, ty = col.b + col.cy * iy, zc = col.c + col.cz * iz;
    lid = tx + (unsigned)g.nt[0] * (ty + (unsigned)g.nt[1] * zc);
  }
  op3d_body<P, TE, MODE, NR, S, op3d_backward<P, MODE, NR, S>(), F>(
      x, y, fac, tB0, tB1, tB2, tD0, tD1, tD2, g, ze, n_free, alpha, lid);
}

// Several patches of one degree in one launch: a static queue of tiles, the
// tiles of patch e numbered tile0..tile0+ntiles-1; workgroup w walks `per_wg`
// consecutive queue entries (w remapped so that each XCD owns a contiguous
// stretch of the queue).  Patch e's vectors start at offset `off` of x and y,
// right-hand sides `stride` entries apart.
template <int P, int TE, int MODE, int NR, typename S>
__global__ void __launch_bounds__((Tile3<P, TE>::NT), (MODE == 1 ? GA_OP3_WAVES_K : GA_OP3_WAVES_M))
op3d_group_kernel(const OpGroupEntry* __restrict__ ents, int nent, const S* __restrict__ x,
                  S* __restrict__ y, long long stride, S alpha, int total, int per_wg,
                  BatchGate gate) {
  const unsigned w = xcd_remap(blockIdx.x, gridDim.x);
  for (int i = 0; i < per_wg; ++i) {
    const int t = (int)w * per_wg + i;
    if (t >= total) return;
    int e = 0;
    while (e + 1 < nent && t >= ents[e + 1].tile0) ++e;
    const OpGroupEntry& d = ents[e];
    bool any = false;
#pragma unroll
    for (int j = 0; j < NR; ++j) any |= batch_active(gate, d.sys, j);
    if (!any) continue;   // uniform over the workgroup (one tile per iteration)
    __syncthreads();  // the previous tile has finished with the LDS
    op3d_body<P, TE, MODE, NR, S, op3d_group_backward<P, MODE, NR>(), S>(x + d.off, y + d.off, (const S*)d.fac, d.tB[0], d.tB[1],
                                             d.tB[2], d.tD[0], d.tD[1], d.tD[2], d.g, d.ze, stride,
                                             alpha, (unsigned)(t - d.tile0));
  }
}


inline int pick_ze(long long ntxy, int nz, int floor_ze) {
  int ze = nz;
  while (ze > floor_ze && ntxy * ((nz + ze - 1) / ze) < 4096) ze = (ze + 1) / 2;
  return ze < 1 ? 1 : ze;
}

// one apply of a 3-D patch: S the arithmetic and vector type, F the storage type of
// the factors (S, or BF16 bit patterns); diag(M) (mode 2) only in FP64
template <int P, typename S, typename F = S>
inline int launch_op3d_p(int mode, int nr, const ga_patch* pt, const S* x, S* y, S alpha,
                         const F* fac, hipStream_t st, const double* gate = nullptr) {
  constexpr int TK = te3_stiff(P), TM = te3_mass(P);
  Geo3 g;
  for (int a = 0; a < 3; ++a) { g.n[a] = pt->n[a]; g.m[a] = pt->m[a]; g.mf[a] = pt->mf[a]; g.lo[a] = pt->lo[a]; }
  const int* nt = mode == 1 ? pt->ntk : pt->ntm;
  g.nt[0] = nt[0];
  g.nt[1] = nt[1];
  const long long ntxy = (long long)nt[0] * nt[1];
  const int ze = op3d_default_ze(mode, pt, sizeof(S) == 4);
  const int nzc = (pt->n[2] + ze - 1) / ze;
  const long long nwg = ntxy * nzc;
  const double* const* B = (mode == 2) ? pt->tabB2 : pt->tabB;
  // deterministic mode: colour classes of tiles that share no coefficient.  Tiles t and
  // t + c along x (or y) are disjoint when c * TE >= TE + P; z ranges when c * ze >= ze + P.
  const int TEk = mode == 1 ? TK : TM;
  // diag(M) (mode 2, patch setup) always takes the ordered launches: the scaling s of
  // the preconditioner is then the same bits on every run
  const bool ordered = pt->deterministic || mode == 2;
  const int cxy = ordered ? 1 + (P + TEk - 1) / TEk : 0;
  const int cz = ordered ? (nzc == 1 ? 1 : 1 + (P + ze - 1) / ze) : 0;
  auto launch = [&](dim3 grid, TileColor col) {
#define GA_OP3(TE, MODE, NRV)                                                                  \
  hipLaunchKernelGGL((op3d_kernel<P, TE, MODE, NRV, S, F>), grid, dim3(Tile3<P, TE>::NT), 0, st, \
                     x, y, fac, B[0], B[1], B[2], pt->tabD[0], pt->tabD[1], pt->tabD[2], g,      \
                     ze, pt->n_free, alpha, gate, col)
    if (mode == 0) {
      if (nr == 1) GA_OP3(TM, 0, 1); else if (nr == 2) GA_OP3(TM, 0, 2); else GA_OP3(TM, 0, 3);
    } else if (mode == 1) {
      if (nr == 1) GA_OP3(TK, 1, 1); else if (nr == 2) GA_OP3(TK, 1, 2); else GA_OP3(TK, 1, 3);
    } else {
      if constexpr (sizeof(S) == 8 && sizeof(F) == 8) GA_OP3(TM, 2, 1);
    }
#undef GA_OP3
  };
  if (nr < 1 || nr > 3) return -1;
  if (mode == 1 && nr > op3d_max_nr(P, 1)) return -1;
  if (mode == 2 && !(sizeof(S) == 8 && sizeof(F) == 8)) return -1;
  if (!cxy) {
    launch(dim3((unsigned)nwg), TileColor{0, 0, 0, 0, 0, 0, 0, 0});
  } else {
    for (int c = 0; c < cz; ++c)
      for (int b = 0; b < cxy; ++b)
        for (int a = 0; a < cxy; ++a) {
          const int nx = (nt[0] - a + cxy - 1) / cxy, ny = (nt[1] - b + cxy - 1) / cxy;
          const int nz = (nzc - c + cz - 1) / cz;
          if (nx <= 0 || ny <= 0 || nz <= 0) continue;
          launch(dim3((unsigned)((long long)nx * ny * nz)), TileColor{cxy, cxy, cz, a, b, c, nx, ny});
        }
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ga
