// Learned initial guess for the stage solves: a 3-layer 3x3x3 convolutional net
// (4 -> 32 -> 32 -> 1 channels, ReLU after the first two layers, zero padding at
// the grid boundary as the homogeneous Dirichlet condition gives) that corrects
// the cubic extrapolation E of the last four solutions H1..H4 of one stage:
//     D0 = H1, D1 = H1 - H2, D2 = H1 - 2H2 + H3, D3 = H1 - 3H2 + 3H3 - H4
//        (backward differences; E = D0 + D1 + D2 + D3 = 4H1 - 6H2 + 4H3 - H4)
//     c_i = D_i / s_i,  s_i = RMS(D_i)       (1 where D_i = 0)
//     guess = E + s_3 * net(c_0, c_1, c_2, c_3).
// Scaling every channel by its own RMS keeps inputs and target of order one,
// although the differences are orders of magnitude below the fields.
//
// Training (on crops):  forward / backward-data / backward-weight / MSE / Adam, with
//   FP32 master weights, activations and gradients.  Crops are channel-major
//   [b][c][S^3]; the convolutions are "valid" and the activations of layers 1 and 2 at
//   positions outside the grid are forced to zero, which makes a crop reproduce the
//   whole-grid net on its interior.  Layer 2's three passes run either in FP32 on the
//   vector units or on MFMA 32x32x16 with BF16 operands and FP32 accumulation; layers
//   1 and 3 run in FP32.
// Inference (whole grid; BF16 inputs, weights and activations; FP32 accumulation),
// three kernels over the same tiles, each staging its input brick in LDS:
//   layer 1 forms the four channels from the FP64 history into the brick and runs
//     on MFMA 32x32x16 (7 k-slices of 4 taps x 4 channels);
//   layer 2 (55,296 of the 63,936 flops per point) runs on MFMA 32x32x16, and in
//     its epilogue two more MFMAs per group form layer 3's per-tap products
//     u[t][p] = sum_c W3[t][c] a2[p][c] (taps as rows), stored as 27 BF16 planes;
//   a last kernel sums u[t] over the 27 tap offsets of each point and forms the
//     guess in FP64.
//   The layer-1 activations are stored channels-last [point][32] (64 bytes per
//   point), the tap planes in 54 bytes per point.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <type_traits>

#include "gnet.h"

namespace ga {

namespace {

constexpr int VB = 256;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

inline unsigned nbk(long long n) {
  long long b = (n + VB - 1) / VB;
  if (b > 65535 * 4) b = 65535 * 4;
  return (unsigned)(b < 1 ? 1 : b);
}

struct Dims {
  int x, y, z;
  __host__ __device__ long long vol() const { return (long long)x * y * z; }
};

__device__ __forceinline__ bool inside(int x, int y, int z, Dims g) {
  return x >= 0 && y >= 0 && z >= 0 && x < g.x && y < g.y && z < g.z;
}

// sq[i] = sum of D_i^2 over the grid -> 1 / s_i
__device__ __forceinline__ double inv_rms(const double* sq, int i, long long n) {
  const double s = sqrt(sq[i] / (double)n);
  return s > 0.0 ? 1.0 / s : 1.0;
}

__device__ __forceinline__ void differences(double h0, double h1, double h2, double h3, double d[4]) {
  d[0] = h0;
  d[1] = h0 - h1;
  d[2] = h0 - 2.0 * h1 + h2;
  d[3] = h0 - 3.0 * h1 + 3.0 * h2 - h3;
}

// ---------------------------------------------------------------- training

// valid convolution of a batch of crops; output o reads input o + (0..2) per axis.
// With org != nullptr, outputs whose grid position org + o + shift lies outside
// the grid are zero.
template <int CI, int CO>
__global__ void __launch_bounds__(VB)
conv_fwd_k(const float* __restrict__ in, Dims di, Dims dout, int nb, const float* __restrict__ W,
           const float* __restrict__ bias, float* __restrict__ out, int relu, Dims grid,
           const int* __restrict__ org, int shift) {
  const long long vi = di.vol(), vo = dout.vol();
  for (long long g = (long long)blockIdx.x * VB + threadIdx.x; g < nb * vo;
       g += (long long)gridDim.x * VB) {
    const long long bi = g / vo, o = g % vo;
    const int ox = (int)(o % dout.x), oy = (int)((o / dout.x) % dout.y),
              oz = (int)(o / ((long long)dout.x * dout.y));
    float* ob = out + bi * CO * vo + o;
    if (org && !inside(org[3 * bi] + ox + shift, org[3 * bi + 1] + oy + shift,
                       org[3 * bi + 2] + oz + shift, grid)) {
#pragma unroll
      for (int c = 0; c < CO; ++c) ob[c * vo] = 0.0f;
      continue;
    }
    float acc[CO];
#pragma unroll
    for (int c = 0; c < CO; ++c) acc[c] = bias[c];
    const float* ib = in + bi * CI * vi;
    for (int t = 0; t < 27; ++t) {
      const long long p = (ox + t % 3) + (long long)di.x * ((oy + (t / 3) % 3) + (long long)di.y * (oz + t / 9));
#pragma unroll 4
      for (int ci = 0; ci < CI; ++ci) {
        const float v = ib[ci * vi + p];
        const float* w = W + (t * CI + ci) * CO;
#pragma unroll
        for (int c = 0; c < CO; ++c) acc[c] += w[c] * v;
      }
    }
#pragma unroll
    for (int c = 0; c < CO; ++c) ob[c * vo] = relu ? fmaxf(acc[c], 0.0f) : acc[c];
  }
}

// gradient w.r.t. the input of a valid convolution, times the ReLU mask of the
// layer that produced that input (act > 0)
template <int CI, int CO>
__global__ void __launch_bounds__(VB)
conv_bwd_data_k(const float* __restrict__ dout, Dims di, Dims dov, int nb,
                const float* __restrict__ W, const float* __restrict__ act, float* __restrict__ din) {
  const long long vi = di.vol(), vo = dov.vol();
  for (long long g = (long long)blockIdx.x * VB + threadIdx.x; g < nb * vi;
       g += (long long)gridDim.x * VB) {
    const long long bi = g / vi, q = g % vi;
    const int qx = (int)(q % di.x), qy = (int)((q / di.x) % di.y), qz = (int)(q / ((long long)di.x * di.y));
    float acc[CI];
#pragma unroll
    for (int c = 0; c < CI; ++c) acc[c] = 0.0f;
    const float* db = dout + bi * CO * vo;
    for (int t = 0; t < 27; ++t) {
      const int ox = qx - t % 3, oy = qy - (t / 3) % 3, oz = qz - t / 9;
      if (ox < 0 || oy < 0 || oz < 0 || ox >= dov.x || oy >= dov.y || oz >= dov.z) continue;
      const long long o = ox + (long long)dov.x * (oy + (long long)dov.y * oz);
      float dv[CO];
#pragma unroll
      for (int co = 0; co < CO; ++co) dv[co] = db[co * vo + o];
#pragma unroll 4
      for (int c = 0; c < CI; ++c) {
        const float* w = W + (t * CI + c) * CO;
        float s = 0.0f;
#pragma unroll
        for (int co = 0; co < CO; ++co) s += w[co] * dv[co];
        acc[c] += s;
      }
    }
    const float* ab = act + bi * CI * vi + q;
    float* ib = din + bi * CI * vi + q;
#pragma unroll
    for (int c = 0; c < CI; ++c) ib[c * vi] = ab[c * vi] > 0.0f ? acc[c] : 0.0f;
  }
}

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// gradient w.r.t. the weights and bias of a valid convolution, in two passes.  Pass 1:
// workgroup (group, chunk) takes input channel ci = blockIdx.x % CI and the G output
// channels co = G (blockIdx.x / CI) + g, which share the 27 input loads of each point,
// and sums the tap products and the bias term over the chunk-th range of `chunk`
// output points of the batch into part[(chunk * CI * CO + co * CI + ci) * 28 + t]
// (t = 27: the bias term).  Pass 2 (conv_bwd_w_finish_k) sums the chunks in order.
template <int CI, int CO, int G>
__global__ void __launch_bounds__(VB)
conv_bwd_w_k(const float* __restrict__ in, Dims di, const float* __restrict__ dout, Dims dov,
             int nb, long long chunk, float* __restrict__ part) {
  const int ci = blockIdx.x % CI, co0 = G * (blockIdx.x / CI);
  const long long vi = di.vol(), vo = dov.vol();
  const long long c0 = (long long)blockIdx.y * chunk, c1 = min(c0 + chunk, nb * vo);
  float acc[G][27], accb[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    accb[g] = 0.0f;
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[g][t] = 0.0f;
  }
  for (long long p = c0 + threadIdx.x; p < c1; p += VB) {
    const long long bi = p / vo, o = p % vo;
    const int ox = (int)(o % dov.x), oy = (int)((o / dov.x) % dov.y), oz = (int)(o / ((long long)dov.x * dov.y));
    float d[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      d[g] = dout[(bi * CO + co0 + g) * vo + o];
      accb[g] += d[g];
    }
    const float* ib = in + (bi * CI + ci) * vi + ox + (long long)di.x * (oy + (long long)di.y * oz);
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const float x = ib[(t % 3) + (long long)di.x * ((t / 3) % 3 + (long long)di.y * (t / 9))];
#pragma unroll
      for (int g = 0; g < G; ++g) acc[g][t] += d[g] * x;
    }
  }
  __shared__ float sh[G][28][VB / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const float v = wsum(acc[g][t]);
      if (lane == 0) sh[g][t][wv] = v;
    }
    const float v = wsum(accb[g]);
    if (lane == 0) sh[g][27][wv] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < G * 28; e += VB) {
    const int g = e / 28, t = e % 28;
    float v = 0.0f;
    for (int w = 0; w < VB / 64; ++w) v += sh[g][t][w];
    part[((long long)blockIdx.y * CI * CO + (co0 + g) * CI + ci) * 28 + t] = v;
  }
}

template <int CI, int CO>
__global__ void __launch_bounds__(VB)
conv_bwd_w_finish_k(const float* __restrict__ part, int nchunk, float* __restrict__ dW,
                    float* __restrict__ dbias) {
  const int j = blockIdx.x * VB + threadIdx.x;
  if (j >= CI * CO * 28) return;
  const int pair = j / 28, t = j % 28, co = pair / CI, ci = pair % CI;
  if (t == 27 && ci != 0) return;
  float s = 0.0f;
  for (int c = 0; c < nchunk; ++c) s += part[((long long)c * CI * CO + pair) * 28 + t];
  if (t < 27) dW[(t * CI + ci) * CO + co] = s;
  else dbias[co] = s;
}

// point chunks of the two-pass weight gradient: about 2048 workgroups in all
constexpr int BWD_W_GROUPS = 2048;

template <int CI, int CO>
void launch_bwd_w(const float* in, Dims di, const float* dout, Dims dov, int nb, float* wpart,
                  float* dW, float* dbias, hipStream_t st) {
  constexpr int G = CO % 4 == 0 ? 4 : 1;   // output channels per workgroup
  constexpr int groups = CI * CO / G;
  const long long npts = nb * dov.vol();
  const int want = BWD_W_GROUPS / groups > 0 ? BWD_W_GROUPS / groups : 1;
  const long long chunk = (npts + want - 1) / want;
  const int nchunk = (int)((npts + chunk - 1) / chunk);
  hipLaunchKernelGGL((conv_bwd_w_k<CI, CO, G>), dim3(groups, nchunk), dim3(VB), 0, st, in, di, dout,
                     dov, nb, chunk, wpart);
  hipLaunchKernelGGL((conv_bwd_w_finish_k<CI, CO>), dim3((CI * CO * 28 + VB - 1) / VB), dim3(VB), 0,
                     st, wpart, nchunk, dW, dbias);
}

// d = 2 (out - tgt) / n; per-block partial sums of (out - tgt)^2
__global__ void __launch_bounds__(VB)
mse_grad_k(const float* __restrict__ out, const float* __restrict__ tgt, long long n,
           float* __restrict__ d, double* __restrict__ part) {
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  for (long long i = (long long)blockIdx.x * VB + threadIdx.x; i < n; i += (long long)gridDim.x * VB) {
    const float e = out[i] - tgt[i];
    d[i] = sc * e;
    s += (double)e * e;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ double sh[VB / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < VB / 64; ++w) t += sh[w];
    part[blockIdx.x] = t;
  }
}

__global__ void adam_k(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * VB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// per-block partial sums of D_i^2, part[i * gridDim.x + block]
__global__ void __launch_bounds__(VB)
diff_norms_k(GnetFields f, long long n, double* __restrict__ part) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // four points per trip with their 16 loads in flight together, added in point order
  const long long stride = (long long)gridDim.x * VB;
  long long i = (long long)blockIdx.x * VB + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double h[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < 4; ++c) h[u][c] = f.h[c][i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double d[4];
      differences(h[u][0], h[u][1], h[u][2], h[u][3], d);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += d[c] * d[c];
    }
  }
  for (; i < n; i += stride) {
    double d[4];
    differences(f.h[0][i], f.h[1][i], f.h[2][i], f.h[3][i], d);
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] += d[c] * d[c];
  }
  __shared__ double sh[4][VB / 64];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double v = acc[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < VB / 64; ++w) t += sh[threadIdx.x][w];
    part[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// crops: in[b][c][S^3] = D_c / s_c around origin org_b (zero outside the grid);
// tgt[b][(S-6)^3] = (X - E) / s_3 on the crop interior
__global__ void __launch_bounds__(VB)
make_batch_k(GnetFields f, Dims grid, const int* __restrict__ org, int S, int nb,
             const double* __restrict__ sq, float* __restrict__ in, float* __restrict__ tgt) {
  const long long vs = (long long)S * S * S;
  const int T = S - 6;
  const long long vt = (long long)T * T * T;
  double is[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) is[c] = inv_rms(sq, c, grid.vol());
  for (long long g = (long long)blockIdx.x * VB + threadIdx.x; g < nb * vs;
       g += (long long)gridDim.x * VB) {
    const long long bi = g / vs, l = g % vs;
    const int lx = (int)(l % S), ly = (int)((l / S) % S), lz = (int)(l / ((long long)S * S));
    const int x = org[3 * bi] + lx, y = org[3 * bi + 1] + ly, z = org[3 * bi + 2] + lz;
    const bool ok = inside(x, y, z, grid);
    const long long p = ok ? x + (long long)grid.x * (y + (long long)grid.y * z) : 0;
    double d[4] = {0.0, 0.0, 0.0, 0.0};
    if (ok) differences(f.h[0][p], f.h[1][p], f.h[2][p], f.h[3][p], d);
#pragma unroll
    for (int c = 0; c < 4; ++c) in[(bi * 4 + c) * vs + l] = (float)(d[c] * is[c]);
    if (lx >= 3 && ly >= 3 && lz >= 3 && lx < S - 3 && ly < S - 3 && lz < S - 3) {
      const double e = d[0] + d[1] + d[2] + d[3];
      const double xv = ok ? f.x[p] : 0.0;
      tgt[bi * vt + (lx - 3) + (long long)T * ((ly - 3) + (long long)T * (lz - 3))] =
          (float)((xv - e) * is[3]);
    }
  }
}

// ---------------------------------------------------------------- training, layer 2 on MFMA
// Layer 2 carries 55,296 of the 63,936 flops per point in each of the forward, the
// backward-data and the backward-weight pass.  In BF16 training these three run on
// MFMA 32x32x16 with BF16 operands (rounded from the FP32 activations, gradients and
// master weights as they are loaded) and FP32 accumulation; activations, gradients
// and the parameter update stay FP32.  MFMA operand layout (one 64-lane wave): lane l
// supplies A[m = l%32][k = 8 (l/32) + i] and B[k = 8 (l/32) + i][n = l%32], i < 8;
// accumulator entry v of lane l is D[8 (v/4) + 4 (l/32) + v%4][l%32].

// W2 for the A operand of the forward (row co, k = ci; the inference layout) and of
// the backward-data pass (row ci, k = co):
//   entry ((t*2 + kc)*64 + lane)*8 + i            = W2[t][16 kc + 8 (lane/32) + i][lane % 32]
//   entry GNET_PACK2 + ((t*2 + kc)*64 + lane)*8 + i = W2[t][lane % 32][16 kc + 8 (lane/32) + i]
__global__ void __launch_bounds__(VB)
pack_w2_train_k(const float* __restrict__ params, __bf16* __restrict__ pk) {
  const int e = blockIdx.x * VB + threadIdx.x;
  if (e >= 2 * GNET_PACK2) return;
  const int which = e / GNET_PACK2, r = e % GNET_PACK2;
  const int i = r % 8, lane = (r / 8) % 64, tk = r / 512, kc = tk % 2, t = tk / 2;
  const int a = 16 * kc + 8 * (lane / 32) + i, b = lane % 32;
  const int ci = which ? b : a, co = which ? a : b;
  pk[e] = (__bf16)params[GNET_W2 + (t * 32 + ci) * 32 + co];
}

// forward of layer 2: wave w of the grid computes the 32 output channels of the 32
// consecutive output points 32 w .. 32 w + 31 of the batch (flattened [b][S2^3]);
// the B operand of tap t and channel slice kc is read from the channel-major a1
// [b][32][S1^3].  Bias, ReLU and the outside-the-grid zeroing as in conv_fwd_k.
__global__ void __launch_bounds__(256)
conv2_train_fwd_k(const float* __restrict__ a1, int S1, int nb, const bf16x8* __restrict__ pk,
                  const float* __restrict__ bias, float* __restrict__ a2, Dims grid,
                  const int* __restrict__ org) {
  const int S2 = S1 - 2;
  const long long vi = (long long)S1 * S1 * S1, vo = (long long)S2 * S2 * S2;
  const int lane = threadIdx.x & 63, n32 = lane & 31, half = lane >> 5;
  const long long g = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + n32;
  const bool valid = g < nb * vo;
  const long long bi = valid ? g / vo : 0, o = valid ? g % vo : 0;
  const int ox = (int)(o % S2), oy = (int)((o / S2) % S2), oz = (int)(o / ((long long)S2 * S2));
  const float* src = a1 + (bi * 32 + 8 * half) * vi + ox + (long long)S1 * (oy + (long long)S1 * oz);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  for (int tr = 0; tr < 9; ++tr) {
    const long long offr = (long long)S1 * (tr % 3 + (long long)S1 * (tr / 3));
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        bf16x8 B;
#pragma unroll
        for (int i = 0; i < 8; ++i) B[i] = (__bf16)src[(16 * kc + i) * vi + offr + kx];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pk[((3 * tr + kx) * 2 + kc) * 64 + lane], B,
                                                       acc, 0, 0, 0);
      }
  }
  if (!valid) return;
  const bool in_grid = inside(org[3 * bi] + ox + 2, org[3 * bi + 1] + oy + 2,
                              org[3 * bi + 2] + oz + 2, grid);
  float* dst = a2 + bi * 32 * vo + o;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int co = 8 * (v / 4) + 4 * half + v % 4;
    dst[co * vo] = in_grid ? fmaxf(acc[v] + bias[co], 0.0f) : 0.0f;
  }
}

// backward-data of layer 2: d1[b][ci][q] = [a1 > 0] sum_{t,co} W2[t][ci][co] d2[b][co][q - o_t]
// over the taps whose output point q - o_t lies in the S2^3 output; wave w computes
// the 32 channels of the 32 input points 32 w .. 32 w + 31 (flattened [b][S1^3])
__global__ void __launch_bounds__(256)
conv2_train_bwd_data_k(const float* __restrict__ d2, int S1, int nb, const bf16x8* __restrict__ pkT,
                       const float* __restrict__ a1, float* __restrict__ d1) {
  const int S2 = S1 - 2;
  const long long vi = (long long)S1 * S1 * S1, vo = (long long)S2 * S2 * S2;
  const int lane = threadIdx.x & 63, n32 = lane & 31, half = lane >> 5;
  const long long g = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + n32;
  const bool valid = g < nb * vi;
  const long long bi = valid ? g / vi : 0, q = valid ? g % vi : 0;
  const int qx = (int)(q % S1), qy = (int)((q / S1) % S1), qz = (int)(q / ((long long)S1 * S1));
  const float* src = d2 + (bi * 32 + 8 * half) * vo;
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  // tap t reads d2 at output point q - o_t (all 16 channel values of the lane); a
  // masked tap reads offset 0 (in bounds) and is zeroed on conversion.  The loads of
  // tap t + 1 are issued before tap t's conversions and MFMAs.
  auto load_tap = [&](int t, float (&v)[16]) -> bool {
    const int ox = qx - t % 3, oy = qy - (t / 3) % 3, oz = qz - t / 9;
    const bool ok = valid && ox >= 0 && ox < S2 && oy >= 0 && oy < S2 && oz >= 0 && oz < S2;
    const long long off = ok ? ox + (long long)S2 * (oy + (long long)S2 * oz) : 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = src[(c / 8 * 16 + c % 8) * vo + off];
    return ok;
  };
  float cur[16], nxt[16];
  bool okc = load_tap(0, cur);
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    bool okn = false;
    if (t + 1 < 27) okn = load_tap(t + 1, nxt);
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      bf16x8 B;
#pragma unroll
      for (int i = 0; i < 8; ++i) B[i] = (__bf16)(okc ? cur[8 * kc + i] : 0.0f);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pkT[(t * 2 + kc) * 64 + lane], B, acc, 0, 0, 0);
    }
    if (t + 1 < 27) {
#pragma unroll
      for (int c = 0; c < 16; ++c) cur[c] = nxt[c];
      okc = okn;
    }
  }
  if (!valid) return;
  const float* ab = a1 + bi * 32 * vi + q;
  float* dst = d1 + bi * 32 * vi + q;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int ci = 8 * (v / 4) + 4 * half + v % 4;
    dst[ci * vi] = ab[ci * vi] > 0.0f ? acc[v] : 0.0f;
  }
}

// backward-weight of layer 2: dW2[t][ci][co] = sum over the batch's output points o
// of a1[b][ci][o + o_t] d2[b][co][o], one 32 x 32 product per tap with the points as
// k, and the bias gradient sum_o d2[b][co][o].
constexpr int TRAIN_PART = 27 * 1024 + 32;   // floats per partial: W2's and b2's gradient

// backward-weight of layer 2 through LDS.  Workgroup (b, zc) of 3 waves sums over
// the output planes oz in [zc * pz, zc * pz + pz) of crop b, in units of 4 output
// rows x 32 output points: d2 of the unit ([co][4 rows][32 points]) and the layer-1
// activations it meets ([ci][6 rows x 3 planes][36 points]) are staged as BF16 in LDS
// with coalesced loads; wave w owns the 9 taps of tap plane kz = w, and for each
// (row, 16-point k-step, ky) reads two aligned 16-byte A windows that the three kx
// taps share (shifted by kx elements with alignbyte).  Partial sums per workgroup go
// to part[b * nzc + zc] (TRAIN_PART floats: 27 taps x [ci][co], then b2's 32), and
// reduce_chunks_k sums them in a fixed order.
constexpr int BW_ROWS = 4;                         // output rows per unit
constexpr int BW_AROW = 96;                        // bytes per staged a1 row (48 BF16)
constexpr int BW_ACH = 18 * BW_AROW + 16;          // bytes per a1 channel (18 rows), padded
constexpr int BW_BCH = BW_ROWS * 64 + 16;          // bytes per d2 channel (4 rows of 32), padded
constexpr int BW_LDS = 32 * BW_ACH + 32 * BW_BCH;  // 64,512 bytes

__device__ __forceinline__ bf16x8 shift_window(const uint4& lo, const uint4& hi, int kx) {
  // elements kx .. kx + 7 of the 16-element window lo:hi
  const unsigned w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  const bool d = kx >= 2;
  const unsigned bs = (kx & 1) * 2;
  unsigned u[5], o[4];
#pragma unroll
  for (int j = 0; j < 5; ++j) u[j] = d ? w[j + 1] : w[j];
#pragma unroll
  for (int j = 0; j < 4; ++j) o[j] = __builtin_amdgcn_alignbyte(u[j + 1], u[j], bs);
  bf16x8 r;
  __builtin_memcpy(&r, o, 16);
  return r;
}

__global__ void __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(2, 2)))
conv2_train_bwd_w_lds_k(const float* __restrict__ a1, const float* __restrict__ d2, int S1, int nb,
                        int pz, int nzc, float* __restrict__ part) {
  __shared__ __align__(16) unsigned char lds[BW_LDS];
  unsigned char* const la = lds;                  // a1 tile
  unsigned char* const lb = lds + 32 * BW_ACH;    // d2 tile
  const int S2 = S1 - 2;
  const long long vi = (long long)S1 * S1 * S1, vo = (long long)S2 * S2 * S2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, n32 = lane & 31, half = lane >> 5;
  const int b = blockIdx.x / nzc, zc = blockIdx.x % nzc;
  const float* a1b = a1 + (long long)b * 32 * vi;
  const float* d2b = d2 + (long long)b * 32 * vo;
  f32x16 acc[9];
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[a][v] = 0.0f;
  float bacc[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) bacc[j] = 0.0f;
  const int oz1 = min(zc * pz + pz, S2);
  for (int oz = zc * pz; oz < oz1; ++oz)
    for (int y0 = 0; y0 < S2; y0 += BW_ROWS)
      for (int x0 = 0; x0 < S2; x0 += 32) {
        // d2: 2048 pairs (co, row r, x pair p), zero outside the output
#pragma unroll
        for (int j = 0; j < 11; ++j) {
          const int pi = tid + 192 * j;
          if (pi < 2048) {
            const int p = pi & 15, r = (pi >> 4) & 3, co = pi >> 6;
            const int y = y0 + r, x = x0 + 2 * p;
            // entries outside the output load offset 0 (in bounds) without a branch and are
            // zeroed by the select, so the loads of all pairs are in flight together
            const bool ok0 = y < S2 && x < S2, ok1 = y < S2 && x + 1 < S2;
            const float* src = d2b + co * vo;
            const long long e = ((long long)oz * S2 + y) * S2 + x;
            const float l0 = src[ok0 ? e : 0], l1 = src[ok1 ? e + 1 : 0];
            const float v0 = ok0 ? l0 : 0.0f, v1 = ok1 ? l1 : 0.0f;
            bacc[j] += v0 + v1;
            const __bf16 h[2] = {(__bf16)v0, (__bf16)v1};
            __builtin_memcpy(lb + co * BW_BCH + r * 64 + 4 * p, h, 4);
          }
        }
        // a1: 10368 pairs (ci, staged row = rr + 6 kz, x pair p), zero outside the crop;
        // 9 batches of 6 pairs per thread, each batch's 12 loads issued before its stores
#pragma unroll 1
        for (int j0 = 0; j0 < 54; j0 += 6) {
          float l0[6], l1[6];
          bool k0[6], k1[6];
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) {
            const int pi = tid + 192 * (j0 + jj);
            const int p = pi % 18, row = (pi / 18) % 18, ci = pi / 324;
            const int rr = row % 6, kz = row / 6;
            const int y = y0 + rr, x = x0 + 2 * p;
            k0[jj] = y < S1 && x < S1;
            k1[jj] = y < S1 && x + 1 < S1;
            const float* src = a1b + ci * vi;
            const long long e = ((long long)(oz + kz) * S1 + y) * S1 + x;
            l0[jj] = src[k0[jj] ? e : 0];
            l1[jj] = src[k1[jj] ? e + 1 : 0];
          }
#pragma unroll
          for (int jj = 0; jj < 6; ++jj) {
            const int pi = tid + 192 * (j0 + jj);
            const int p = pi % 18, row = (pi / 18) % 18, ci = pi / 324;
            const __bf16 h[2] = {(__bf16)(k0[jj] ? l0[jj] : 0.0f), (__bf16)(k1[jj] ? l1[jj] : 0.0f)};
            __builtin_memcpy(la + ci * BW_ACH + row * BW_AROW + 4 * p, h, 4);
          }
        }
        __syncthreads();
        // wave w: taps (kx, ky, kz = w); lane supplies A[ci = n32][8 half + i] and
        // B[8 half + i][co = n32] of the k-step's 16 points
#pragma unroll
        for (int r = 0; r < BW_ROWS; ++r)
#pragma unroll
          for (int ks = 0; ks < 2; ++ks) {
            const int xo = 16 * ks + 8 * half;
            bf16x8 B;
            {
              const uint4 raw = *reinterpret_cast<const uint4*>(lb + n32 * BW_BCH + r * 64 + 2 * xo);
              __builtin_memcpy(&B, &raw, 16);
            }
#pragma unroll
            for (int ky = 0; ky < 3; ++ky) {
              const unsigned char* ap = la + n32 * BW_ACH + (r + ky + 6 * w) * BW_AROW + 2 * xo;
              const uint4 lo = *reinterpret_cast<const uint4*>(ap);
              const uint4 hi = *reinterpret_cast<const uint4*>(ap + 16);
#pragma unroll
              for (int kx = 0; kx < 3; ++kx)
                acc[3 * ky + kx] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(shift_window(lo, hi, kx), B,
                                                                            acc[3 * ky + kx], 0, 0, 0);
            }
          }
        __syncthreads();
      }
  float* pc = part + (long long)blockIdx.x * TRAIN_PART;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    float* dst = pc + (9 * w + a) * 1024 + n32;
#pragma unroll
    for (int v = 0; v < 16; ++v) dst[(8 * (v / 4) + 4 * half + v % 4) * 32] = acc[a][v];
  }
#pragma unroll
  for (int j = 0; j < 11; ++j) {
    const float t = wsum(bacc[j]);
    const int co = w + 3 * j;
    if (lane == 0 && co < 32) pc[27 * 1024 + co] = t;
  }
}

// out[j] = sum over c < nchunk of part[c * n + j]: a workgroup takes 64 consecutive j,
// its four waves a quarter of the chunks each (in order), and the four partial sums
// are added in wave order
__global__ void __launch_bounds__(VB)
reduce_chunks_k(const float* __restrict__ part, long long nchunk, int n, float* __restrict__ out) {
  __shared__ float sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const long long q = (nchunk + 3) / 4, c0 = w * q, c1 = min(c0 + q, nchunk);
  float s = 0.0f;
  if (j < n) {
#pragma unroll 8
    for (long long c = c0; c < c1; ++c) s += part[c * n + j];
  }
  sh[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) out[j] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

// ---------------------------------------------------------------- inference

// One buffer of BF16 weights:
//   [0, GNET_PACK2): W2 for the MFMA A operand, entry ((t*2 + kc)*64 + lane)*8 + i
//     holds W2[t][ci = 16 kc + 8 (lane/32) + i][co = lane % 32];
//   then GNET_PACK1: W1 likewise, entry (j*64 + lane)*8 + i holds W1[t][ci][co] with
//     t = 4 j + 2 (lane/32) + i/4, ci = i % 4, co = lane % 32 (zero for t = 27);
//   then GNET_PACK3: W3 for the A operand of layer 3's per-tap products, entry
//     (s*64 + lane)*8 + i holds W3[t = lane % 32][layer3_channel(s, lane / 32, i)]
//     (zero for t >= 27).
// Channel that k index 8 h + i of k-slice s stands for in layer 3's products: lane
// half h of layer 2's accumulators holds channels 8 q + 4 h + j (q, j < 4) as entries
// 4 q + j, so slice s takes entries 8 s .. 8 s + 7 of each lane as they are
__host__ __device__ constexpr int layer3_channel(int s, int h, int i) {
  return 8 * (2 * s + i / 4) + 4 * h + i % 4;
}

__global__ void pack_w_k(const float* __restrict__ params, __bf16* __restrict__ pk) {
  const int e = blockIdx.x * VB + threadIdx.x;
  if (e < GNET_PACK2) {
    const int i = e % 8, lane = (e / 8) % 64, kc = (e / 512) % 2, t = e / 1024;
    const int ci = 16 * kc + 8 * (lane / 32) + i, co = lane % 32;
    pk[e] = (__bf16)params[GNET_W2 + (t * 32 + ci) * 32 + co];
  } else if (e < GNET_PACK2 + GNET_PACK1) {
    const int r = e - GNET_PACK2;
    const int i = r % 8, lane = (r / 8) % 64, j = r / 512;
    const int t = 4 * j + 2 * (lane / 32) + i / 4, ci = i % 4, co = lane % 32;
    pk[e] = t < 27 ? (__bf16)params[GNET_W1 + (t * 4 + ci) * 32 + co] : (__bf16)0.0f;
  } else if (e < GNET_PACK) {
    const int r = e - GNET_PACK2 - GNET_PACK1;
    const int i = r % 8, lane = (r / 8) % 64, sl = r / 512;
    const int t = lane % 32, ci = layer3_channel(sl, lane / 32, i);
    pk[e] = t < 27 ? (__bf16)params[GNET_W3 + t * 32 + ci] : (__bf16)0.0f;
  }
}

// Workgroup tile of every inference kernel: 16 (x) x 8 (y) x 4 (z) output points; its
// input brick with a one-point halo is 18 x 10 x 6 points.  Wave w owns z-plane w of
// the tile; an MFMA 32x32x16 covers 32 output channels x 32 points (16 x by 2 y).
constexpr int TX = 16, TY = 8, TZ = 4, HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HP = HX * HY * HZ;

__device__ __forceinline__ unsigned xcd_tile(unsigned bid, unsigned nwg) {
  // consecutive tiles (which share halo data) on the same XCD
  const unsigned nx = 8, per = nwg / nx, rem = nwg % nx;
  const unsigned xcd = bid % nx, loc = bid / nx;
  const unsigned base = xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per;
  return base + loc;
}

// ReLU(acc + bias) of 4 groups of 32 points to BF16 channels-last rows of 32
// channels (accumulator v of lane l holds channel 8 (v/4) + 4 (l/32) + v%4 of point
// l%32), points outside the grid skipped
__device__ __forceinline__ void store_act(const f32x16 (&acc)[4], const float* __restrict__ bias,
                                          __bf16* __restrict__ out, Dims g, int x0, int y0, int oz,
                                          int lx, int ly, int half) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ox = x0 + lx, oy = y0 + 2 * r + ly;
    if (!inside(ox, oy, oz, g)) continue;
    __bf16* dst = out + (ox + (long long)g.x * (oy + (long long)g.y * oz)) * 32;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c0 = 8 * q + 4 * half;
      bf16x4 o4;
#pragma unroll
      for (int i = 0; i < 4; ++i) o4[i] = (__bf16)fmaxf(acc[r][4 * q + i] + bias[c0 + i], 0.0f);
      *reinterpret_cast<bf16x4*>(dst + c0) = o4;
    }
  }
}

// Stage a brick of 32-channel BF16 activations (64 bytes per point, zero outside the
// grid) with every load of a thread in flight before the first LDS store; 16-byte
// channel chunk c of brick point n goes to slot c ^ ((n >> 1) & 3)
__device__ __forceinline__ void stage_act_brick(const uint4* __restrict__ src, Dims g, int x0,
                                                int y0, int z0, uint4* brick, int tid) {
  constexpr int NE = (HP * 4 + 255) / 256;
  uint4 v[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * 256, n = e >> 2, c = e & 3;
    const int hx = n % HX, hy = (n / HX) % HY, hz = n / (HX * HY);
    const int x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 - 1 + hz;
    // points outside the grid load chunk c of point 0 (in bounds) without a branch; the
    // select zeroes them
    const bool in = e < HP * 4 && inside(x, y, z, g);
    const uint4 raw = src[(in ? x + (long long)g.x * (y + (long long)g.y * z) : 0) * 4 + c];
    v[k] = in ? raw : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int e = tid + k * 256, n = e >> 2, c = e & 3;
    if (e < HP * 4) brick[n * 4 + (c ^ ((n >> 1) & 3))] = v[k];
  }
}

// layer 1 on MFMA.  The brick holds the four input channels D_c / s_c of each point
// as BF16 (8 bytes per point), formed from the FP64 history (zero outside the grid);
// the 108 products per output channel (27 taps x 4 channels) are 7 k-slices of 4 taps.
__global__ void __launch_bounds__(256)
conv1_mfma_k(GnetFields f, Dims g, const double* __restrict__ sq, const bf16x8* __restrict__ wpk,
             const float* __restrict__ bias, __bf16* __restrict__ a1, int ntx, int nty) {
  __shared__ uint2 brick[HP];
  const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int tid = threadIdx.x;
  const long long vol = g.vol();
  double is[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) is[c] = inv_rms(sq, c, vol);
  // every history load of a thread in flight before the first LDS store
  constexpr int NE = (HP + 255) / 256;
  double hv[NE][4];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int n = tid + k * 256;
    const int hx = n % HX, hy = (n / HX) % HY, hz = n / (HX * HY);
    const int x = x0 - 1 + hx, y = y0 - 1 + hy, z = z0 - 1 + hz;
    const bool in = n < HP && inside(x, y, z, g);
    const long long p = in ? x + (long long)g.x * (y + (long long)g.y * z) : 0;
    // points outside the grid load point 0 (in bounds) without a branch; the select
    // zeroes them
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double h = f.h[c][p];
      hv[k][c] = in ? h : 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    const int n = tid + k * 256;
    if (n >= HP) continue;
    double d[4];
    differences(hv[k][0], hv[k][1], hv[k][2], hv[k][3], d);
    bf16x4 v;
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = (__bf16)(float)(d[c] * is[c]);
    __builtin_memcpy(&brick[n], &v, 8);
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int n32 = lane & 31, half = lane >> 5, lx = n32 & 15, ly = n32 >> 4;
  f32x16 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[r][v] = 0.0f;
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const bf16x8 A = wpk[j * 64 + lane];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint2 raw[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = 4 * j + 2 * half + h;
        raw[h] = make_uint2(0u, 0u);
        if (t < 27) {
          const int dx = t % 3, dy = (t / 3) % 3, dz = t / 9;
          raw[h] = brick[((w + dz) * HY + (2 * r + ly + dy)) * HX + (lx + dx)];
        }
      }
      bf16x8 B;
      __builtin_memcpy(&B, raw, 16);
      acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[r], 0, 0, 0);
    }
  }
  store_act(acc, bias, a1, g, x0, y0, z0 + w, lx, ly, half);
}

// layer 2 on MFMA.  The brick holds the 32 layer-1 channels of each point (BF16,
// 64 bytes); 16-byte channel chunk c of brick point n sits at slot c ^ ((n >> 1) & 3)
// so that 8 consecutive points read by one LDS phase hit distinct banks.  Each MFMA
// covers one 16-channel slice of one tap: 54 MFMAs per group of 32 points.
__global__ void __launch_bounds__(256)
conv2_mfma_k(const uint4* __restrict__ a1, Dims g, const bf16x8* __restrict__ wpk,
             const float* __restrict__ bias, const bf16x8* __restrict__ w3pk,
             __bf16* __restrict__ u, int ntx, int nty) {
  __shared__ uint4 brick[HP * 4];
  const unsigned tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int tid = threadIdx.x;
  stage_act_brick(a1, g, x0, y0, z0, brick, tid);
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int n32 = lane & 31, half = lane >> 5, lx = n32 & 15, ly = n32 >> 4;
  f32x16 acc[4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[r][v] = 0.0f;
  // k-steps in column order: for each (dz, dx, channel slice kc) the 12 MFMAs of the
  // three dy taps and four point groups read 9 brick rows (rows 2 r + ly + dy, which
  // the groups share across dy) and 3 weight fragments; the next column's operands
  // are read before this column's MFMAs are issued
  auto load_col = [&](int cs, bf16x8 (&A)[3], bf16x8 (&B)[9]) {
    const int kc = cs & 1, dx = (cs >> 1) % 3, dz = (cs >> 1) / 3;
    const int c = kc * 2 + half;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) A[dy] = wpk[((9 * dz + 3 * dy + dx) * 2 + kc) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      const int n = ((w + dz) * HY + (ly + m)) * HX + (lx + dx);
      const uint4 raw = brick[n * 4 + (c ^ ((n >> 1) & 3))];
      __builtin_memcpy(&B[m], &raw, 16);
    }
  };
  // point groups with a row inside the grid (the last tile along y holds one row), and
  // waves whose z-plane lies outside the grid (the last tile along z holds one plane)
  // skip their MFMAs: the test is uniform over the wave, and no barrier follows
  const int ngr = max(0, min(4, (g.y - y0 + 1) / 2));
  if (z0 + w >= g.z) return;
  // the loop is compiled once for four groups (every tile but the last along y) and
  // once with the group test (the last), so the common case keeps a branch-free body
  auto run = [&](auto full) {
    auto mma_col = [&](const bf16x8 (&A)[3], const bf16x8 (&B)[9]) {
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (decltype(full)::value || r < ngr)
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[dy], B[2 * r + dy], acc[r], 0, 0, 0);
    };
    bf16x8 A0[3], A1[3], B0[9], B1[9];
    load_col(0, A0, B0);
    for (int cs = 0; cs < 18; cs += 2) {
      load_col(cs + 1, A1, B1);
      mma_col(A0, B0);
      if (cs + 2 < 18) load_col(cs + 2, A0, B0);
      mma_col(A1, B1);
    }
  };
  if (ngr == 4) run(std::true_type{});
  else run(std::false_type{});
  // layer 3's per-tap products of the tile's points, u[t][p] = sum_c W3[t][c] a2[p][c]:
  // the BF16 activations (bias, ReLU) of each group are the B operand of two MFMAs
  // (k-slice s takes accumulator entries 8 s .. 8 s + 7, see layer3_channel) whose
  // rows are the taps; u is stored as 27 BF16 planes over the grid
  const bf16x8 A3[2] = {w3pk[lane], w3pk[64 + lane]};
  const long long vol = g.vol();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (r >= ngr) continue;
    bf16x8 B3[2];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ch = 8 * (v / 4) + 4 * half + v % 4;
      B3[v / 8][v % 8] = (__bf16)fmaxf(acc[r][v] + bias[ch], 0.0f);
    }
    f32x16 ut;
#pragma unroll
    for (int v = 0; v < 16; ++v) ut[v] = 0.0f;
    ut = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3[0], B3[0], ut, 0, 0, 0);
    ut = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A3[1], B3[1], ut, 0, 0, 0);
    const int ox = x0 + lx, oy = y0 + 2 * r + ly, oz = z0 + w;
    if (!inside(ox, oy, oz, g)) continue;
    const long long p = ox + (long long)g.x * (oy + (long long)g.y * oz);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int t = 8 * (v / 4) + 4 * half + v % 4;   // output row of entry v
      if (t < 27) u[t * vol + p] = (__bf16)ut[v];
    }
  }
}

// layer 3's sum over the taps and the guess: X[q] = E + s_3 (b3 + sum_t u[t][q + o_t]),
// o_t the offset of tap t (zero padding: taps outside the grid are left out); each
// plane is read once over the grid, coalesced.  I is the type of the point index
// (32-bit while the grid has fewer than 2^32 points: no 64-bit division).
template <typename I>
__global__ void __launch_bounds__(VB)
layer3_gather_k(const __bf16* __restrict__ u, GnetFields f, Dims g, const double* __restrict__ sq,
                const float* __restrict__ bias, double* __restrict__ X) {
  const long long v = g.vol(), sy = g.x, sz = (long long)g.x * g.y;
  const double s3 = 1.0 / inv_rms(sq, 3, v);
  const I gx = (I)g.x, gy = (I)g.y;
  for (long long o = (long long)blockIdx.x * VB + threadIdx.x; o < v; o += (long long)gridDim.x * VB) {
    const I io = (I)o, row = io / gx;
    const int ox = (int)(io - row * gx), oy = (int)(row % gy), oz = (int)(row / gy);
    const bool in[3][3] = {{ox > 0, true, ox + 1 < g.x}, {oy > 0, true, oy + 1 < g.y},
                           {oz > 0, true, oz + 1 < g.z}};
    // a tap outside the grid reads the point itself (in bounds) and is zeroed by the
    // select, so all 27 loads are issued without a branch
    float tap[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      const int dx = t % 3, dy = (t / 3) % 3, dz = t / 9;
      const bool ok = in[0][dx] && in[1][dy] && in[2][dz];
      const long long off = ok ? (dx - 1) + (dy - 1) * sy + (dz - 1) * sz : 0;
      const float w = (float)u[t * v + o + off];
      tap[t] = ok ? w : 0.0f;
    }
    float acc = bias[0];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc += tap[t];
    const double e = 4.0 * f.h[0][o] - 6.0 * f.h[1][o] + 4.0 * f.h[2][o] - f.h[3][o];
    X[o] = e + s3 * (double)acc;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

static Dims cube(int s) { return Dims{s, s, s}; }

void gnet_forward_batch(const float* params, const float* in, int nb, int S, const int* grid3,
                        const int* org_dev, float* a1, float* a2, float* out, void* tpk,
                        hipStream_t st) {
  const int S1 = S - 2, S2 = S - 4, S3 = S - 6;
  const Dims g{grid3[0], grid3[1], grid3[2]};
  hipLaunchKernelGGL((conv_fwd_k<4, 32>), dim3(nbk((long long)nb * S1 * S1 * S1)), dim3(VB), 0, st,
                     in, cube(S), cube(S1), nb, params + GNET_W1, params + GNET_B1, a1, 1, g,
                     org_dev, 1);
  if (tpk) {
    hipLaunchKernelGGL(pack_w2_train_k, dim3((2 * GNET_PACK2 + VB - 1) / VB), dim3(VB), 0, st, params,
                       (__bf16*)tpk);
    const long long waves = ((long long)nb * S2 * S2 * S2 + 31) / 32;
    hipLaunchKernelGGL(conv2_train_fwd_k, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, a1, S1,
                       nb, (const bf16x8*)tpk, params + GNET_B2, a2, g, org_dev);
  } else {
    hipLaunchKernelGGL((conv_fwd_k<32, 32>), dim3(nbk((long long)nb * S2 * S2 * S2)), dim3(VB), 0, st,
                       a1, cube(S1), cube(S2), nb, params + GNET_W2, params + GNET_B2, a2, 1, g,
                       org_dev, 2);
  }
  hipLaunchKernelGGL((conv_fwd_k<32, 1>), dim3(nbk((long long)nb * S3 * S3 * S3)), dim3(VB), 0, st,
                     a2, cube(S2), cube(S3), nb, params + GNET_W3, params + GNET_B3, out, 0, g,
                     (const int*)nullptr, 0);
}

// output planes per workgroup of the BF16 backward-weight pass: one, unless the batch
// has more than 1024 planes in all
static void bwd_w_planes(int nb, int S, int* pz, int* nzc) {
  const int S2 = S - 4;
  const long long planes = (long long)nb * S2;
  *pz = (int)std::max<long long>(1, (planes + 1023) / 1024);
  *nzc = (S2 + *pz - 1) / *pz;
}

long long gnet_train_part_floats(int nb, int S) {
  int pz, nzc;
  bwd_w_planes(nb, S, &pz, &nzc);
  return (long long)nb * nzc * TRAIN_PART;
}

// at most BWD_W_GROUPS / (CI CO / G) chunks of CI CO partials of 28 floats, G <= 4
long long gnet_train_wpart_floats() { return (long long)BWD_W_GROUPS * 4 * 28; }

void gnet_backward_batch(const float* params, const float* in, int nb, int S, const float* a1,
                         const float* a2, const float* d3, float* d2, float* d1, float* grad,
                         const void* tpk, float* part, float* wpart, hipStream_t st) {
  const int S1 = S - 2, S2 = S - 4, S3 = S - 6;
  launch_bwd_w<32, 1>(a2, cube(S2), d3, cube(S3), nb, wpart, grad + GNET_W3, grad + GNET_B3, st);
  hipLaunchKernelGGL((conv_bwd_data_k<32, 1>), dim3(nbk((long long)nb * S2 * S2 * S2)), dim3(VB), 0,
                     st, d3, cube(S2), cube(S3), nb, params + GNET_W3, a2, d2);
  if (tpk) {
    int pz, nzc;
    bwd_w_planes(nb, S, &pz, &nzc);
    hipLaunchKernelGGL(conv2_train_bwd_w_lds_k, dim3((unsigned)(nb * nzc)), dim3(192), 0, st, a1, d2,
                       S1, nb, pz, nzc, part);
    // W2's and b2's gradients are contiguous in the parameter layout
    hipLaunchKernelGGL(reduce_chunks_k, dim3((TRAIN_PART + 63) / 64), dim3(VB), 0, st, part,
                       (long long)nb * nzc, TRAIN_PART, grad + GNET_W2);
    const long long wd = ((long long)nb * S1 * S1 * S1 + 31) / 32;
    hipLaunchKernelGGL(conv2_train_bwd_data_k, dim3((unsigned)((wd + 3) / 4)), dim3(256), 0, st, d2,
                       S1, nb, (const bf16x8*)tpk + GNET_PACK2 / 8, a1, d1);
  } else {
    launch_bwd_w<32, 32>(a1, cube(S1), d2, cube(S2), nb, wpart, grad + GNET_W2, grad + GNET_B2, st);
    hipLaunchKernelGGL((conv_bwd_data_k<32, 32>), dim3(nbk((long long)nb * S1 * S1 * S1)), dim3(VB),
                       0, st, d2, cube(S1), cube(S2), nb, params + GNET_W2, a1, d1);
  }
  launch_bwd_w<4, 32>(in, cube(S), d1, cube(S1), nb, wpart, grad + GNET_W1, grad + GNET_B1, st);
}

void gnet_mse_grad(const float* out, const float* tgt, long long n, float* d, double* part,
                   int nparts, hipStream_t st) {
  hipLaunchKernelGGL(mse_grad_k, dim3(nparts), dim3(VB), 0, st, out, tgt, n, d, part);
}

void gnet_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
               float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(adam_k, dim3((n + VB - 1) / VB), dim3(VB), 0, st, p, m, v, g, n, lr, b1, b2,
                     eps, c1, c2);
}

void gnet_diff_norms(GnetFields f, long long n, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(diff_norms_k, dim3(nparts), dim3(VB), 0, st, f, n, part);
}

void gnet_make_batch(GnetFields f, const int* grid3, const int* org_dev, int S, int nb,
                     const double* sq, float* in, float* tgt, hipStream_t st) {
  hipLaunchKernelGGL(make_batch_k, dim3(nbk((long long)nb * S * S * S)), dim3(VB), 0, st, f,
                     Dims{grid3[0], grid3[1], grid3[2]}, org_dev, S, nb, sq, in, tgt);
}

void gnet_pack_bf16(const float* params, void* wpk, hipStream_t st) {
  hipLaunchKernelGGL(pack_w_k, dim3((GNET_PACK + VB - 1) / VB), dim3(VB), 0, st, params,
                     (__bf16*)wpk);
}

void gnet_infer_grid(const float* params, const void* wpk, GnetFields f, const int* grid3,
                     const double* sq, void* a1, void* a2, double* X, hipStream_t st) {
  const Dims g{grid3[0], grid3[1], grid3[2]};
  const int ntx = (g.x + TX - 1) / TX, nty = (g.y + TY - 1) / TY, ntz = (g.z + TZ - 1) / TZ;
  const dim3 grid((unsigned)(ntx * nty * ntz));
  const __bf16* pk = (const __bf16*)wpk;
  hipLaunchKernelGGL(conv1_mfma_k, grid, dim3(256), 0, st, f, g, sq,
                     (const bf16x8*)(pk + GNET_PACK2), params + GNET_B1, (__bf16*)a1, ntx, nty);
  hipLaunchKernelGGL(conv2_mfma_k, grid, dim3(256), 0, st, (const uint4*)a1, g,
                     (const bf16x8*)pk, params + GNET_B2, (const bf16x8*)(pk + GNET_PACK2 + GNET_PACK1),
                     (__bf16*)a2, ntx, nty);
  if (g.vol() < (1ll << 32))
    hipLaunchKernelGGL(layer3_gather_k<unsigned>, dim3(nbk(g.vol())), dim3(VB), 0, st,
                       (const __bf16*)a2, f, g, sq, params + GNET_B3, X);
  else
    hipLaunchKernelGGL(layer3_gather_k<unsigned long long>, dim3(nbk(g.vol())), dim3(VB), 0, st,
                       (const __bf16*)a2, f, g, sq, params + GNET_B3, X);
}

}  // namespace ga
