// Learned initial guess: parameter layout and launchers (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace ga {

// FP32 parameters, tap-major: W1[27][4][32] b1[32] W2[27][32][32] b2[32] W3[27][32] b3[1];
// tap t = 9 kz + 3 ky + kx, weight W[t][ci][co] multiplies in[z+kz-1][y+ky-1][x+kx-1][ci]
constexpr int GNET_W1 = 0;
constexpr int GNET_B1 = GNET_W1 + 27 * 4 * 32;
constexpr int GNET_W2 = GNET_B1 + 32;
constexpr int GNET_B2 = GNET_W2 + 27 * 32 * 32;
constexpr int GNET_W3 = GNET_B2 + 32;
constexpr int GNET_B3 = GNET_W3 + 27 * 32;
constexpr int GNET_NPARAM = GNET_B3 + 1;   // 32033
// BF16 inference weights, one buffer: W2 packed for the MFMA A operand, then W1 packed
// likewise (7 k-slices of 4 taps x 4 channels, the 28th tap zero), then W3 packed as
// the A operand of the per-tap products of layer 3 (taps as rows, 2 channel slices)
constexpr int GNET_PACK2 = 27 * 2 * 64 * 8;
constexpr int GNET_PACK1 = 7 * 64 * 8;
constexpr int GNET_PACK3 = 2 * 64 * 8;
constexpr int GNET_PACK = GNET_PACK2 + GNET_PACK1 + GNET_PACK3;  // bf16 entries

// four history fields (newest first) and the solution they are paired with
struct GnetFields {
  const double* h[4];
  const double* x;
};

// training (channel-major crops [b][c][S^3], valid convolutions; activations of
// layers 1-2 at positions outside the grid are zero, as with per-layer zero padding).
// FP32 throughout when tpk is null; otherwise layer 2's three passes run on BF16 MFMA
// with FP32 accumulation: tpk holds 2 * GNET_PACK2 BF16 entries (16-byte aligned),
// packed by the forward from params, and part gnet_train_part_floats(nb, S) floats of
// layer 2's backward-weight partial sums.  wpart: gnet_train_wpart_floats() floats of
// the FP32 weight gradients' partial sums.  Every sum is taken in a fixed order.
void gnet_forward_batch(const float* params, const float* in, int nb, int S, const int* grid3,
                        const int* org_dev, float* a1, float* a2, float* out, void* tpk,
                        hipStream_t st);
void gnet_backward_batch(const float* params, const float* in, int nb, int S, const float* a1,
                         const float* a2, const float* d3, float* d2, float* d1, float* grad,
                         const void* tpk, float* part, float* wpart, hipStream_t st);
long long gnet_train_part_floats(int nb, int S);
long long gnet_train_wpart_floats();
void gnet_mse_grad(const float* out, const float* tgt, long long n, float* d, double* part,
                   int nparts, hipStream_t st);
void gnet_adam(float* p, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
               float eps, float c1, float c2, hipStream_t st);
// partial sums of the squared backward differences D_0..D_3 of the history,
// part[c * nparts + block]
void gnet_diff_norms(GnetFields f, long long n, double* part, int nparts, hipStream_t st);
void gnet_make_batch(GnetFields f, const int* grid3, const int* org_dev, int S, int nb,
                     const double* sq, float* in, float* tgt, hipStream_t st);

// inference on the whole grid (BF16 inputs, weights and activations, FP32
// accumulation): X = E + s_3 * net(D / s), sq[c] = sum of D_c^2; scratch a1 of 64
// bytes per grid point (layer-1 activations), a2 of 54 (layer 3's tap planes)
void gnet_pack_bf16(const float* params, void* wpk, hipStream_t st);
void gnet_infer_grid(const float* params, const void* wpk, GnetFields f, const int* grid3,
                     const double* sq, void* a1, void* a2, double* X, hipStream_t st);

}  // namespace ga
