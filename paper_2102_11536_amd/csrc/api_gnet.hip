// C ABI of the learned initial guess: net handles, training crops, forward/gradient
// (FP32, or layer 2 on BF16 MFMA) and Adam, BF16 whole-grid inference.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "ga_internal.h"
#include "gnet.h"
#include "kernels.h"

using namespace ga;

namespace {

constexpr int MSE_PARTS = 256;

int grow(void** p, size_t* have, size_t need) {
  if (*have >= need) return GA_OK;
  if (*p) hipFree(*p);
  *p = nullptr;
  *have = 0;
  int rc = dalloc(p, need);
  if (rc) return rc;
  *have = need;
  return GA_OK;
}

// training buffers: a1 [nb][32][S1^3], a2 [nb][32][S2^3], out/d3 [nb][S3^3],
// d2 like a2, d1 like a1, the weight gradients' partial sums; for BF16 training
// also the packed W2 (first, 16-byte aligned) and layer 2's partial sums
struct TrainBufs {
  float *a1, *a2, *out, *d3, *d2, *d1, *wpart;
  void* tpk = nullptr;
  float* part = nullptr;
};

int train_bufs(ga_gnet* net, int nb, int S, TrainBufs* b) {
  const size_t v1 = (size_t)(S - 2) * (S - 2) * (S - 2), v2 = (size_t)(S - 4) * (S - 4) * (S - 4),
               v3 = (size_t)(S - 6) * (S - 6) * (S - 6);
  const size_t n1 = (size_t)nb * 32 * v1, n2 = (size_t)nb * 32 * v2, n3 = (size_t)nb * v3;
  const bool bf = net->train_prec == GA_BF16;
  const size_t npk = bf ? 2 * GNET_PACK2 * sizeof(short) : 0;   // a multiple of 16 bytes
  const size_t npart = bf ? (size_t)gnet_train_part_floats(nb, S) : 0;
  const size_t nw = (size_t)gnet_train_wpart_floats();
  int rc = grow((void**)&net->tw, &net->tw_bytes,
                npk + (npart + nw + 2 * n1 + 2 * n2 + 2 * n3) * sizeof(float));
  if (rc) return rc;
  char* base = (char*)net->tw;
  if (bf) b->tpk = base;
  float* q = (float*)(base + npk);
  if (bf) { b->part = q; q += npart; }
  b->wpart = q; q += nw;
  b->a1 = q; q += n1;
  b->a2 = q; q += n2;
  b->out = q; q += n3;
  b->d3 = q; q += n3;
  b->d2 = q; q += n2;
  b->d1 = q;
  return GA_OK;
}

int check_crops(int nb, int S, const int* grid3, const int* org) {
  if (nb < 1 || S < 7 || S > 512) { set_error("need nb >= 1 and 7 <= S <= 512"); return GA_EINVAL; }
  if (!grid3 || !org) { set_error("null grid or origins"); return GA_EINVAL; }
  for (int a = 0; a < 3; ++a)
    if (grid3[a] < 1) { set_error("bad grid"); return GA_EINVAL; }
  for (int b = 0; b < nb; ++b)
    for (int a = 0; a < 3; ++a) {
      const int o = org[3 * b + a];
      if (o < -3 || o + S - 3 > grid3[a]) {
        set_error("crop target region outside the grid");
        return GA_EINVAL;
      }
    }
  return GA_OK;
}

int upload_origins(ga_gnet* net, int nb, const int* org, hipStream_t st) {
  if (net->org_cap < nb) {
    if (net->org) {
      GA_TRY_HIP(hipStreamSynchronize(st));
      hipFree(net->org);
      net->org = nullptr;
    }
    int rc = dalloc((void**)&net->org, (size_t)nb * 3 * sizeof(int));
    if (rc) return rc;
    net->org_cap = nb;
  }
  // the previous batch may still read the buffer
  GA_TRY_HIP(hipStreamSynchronize(st));
  GA_TRY_HIP(hipMemcpy(net->org, org, (size_t)nb * 3 * sizeof(int), hipMemcpyHostToDevice));
  return GA_OK;
}

int pack_if_needed(ga_gnet* net, hipStream_t st) {
  if (net->packed) return GA_OK;
  gnet_pack_bf16(net->params, net->wpk, st);
  net->packed = true;
  return check_launch(0, "net weight packing");
}

}  // namespace

namespace ga {

int gnet_guess(ga_gnet* net, ga_patch* pt, const double* const* h, double* X, hipStream_t st) {
  const size_t n = pt->n_free;
  int rc = grow(&net->iw, &net->iw_bytes, 2 * n * 32 * sizeof(short));
  if (rc) return rc;
  if ((rc = pack_if_needed(net, st))) return rc;
  GnetFields f{{h[0], h[1], h[2], h[3]}, nullptr};
  gnet_diff_norms(f, (long long)n, net->part, RED_BLOCKS, st);
  launch_sum_partials(4, net->part, net->scal, st);
  char* a1 = (char*)net->iw;
  gnet_infer_grid(net->params, net->wpk, f, pt->mf, net->scal, a1, a1 + n * 64, X, st);
  return check_launch(0, "learned guess");
}

}  // namespace ga

extern "C" {

int ga_gnet_create(const float* params_host, ga_gnet** out) {
  if (!out) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  ga_gnet* net = new ga_gnet();
  int rc;
  if ((rc = dalloc((void**)&net->params, GNET_NPARAM * sizeof(float))) ||
      (rc = dalloc((void**)&net->m, GNET_NPARAM * sizeof(float))) ||
      (rc = dalloc((void**)&net->v, GNET_NPARAM * sizeof(float))) ||
      (rc = dalloc(&net->wpk, GNET_PACK * 2)) ||
      (rc = dalloc((void**)&net->scal, 8 * sizeof(double))) ||
      (rc = dalloc((void**)&net->part, (size_t)4 * RED_BLOCKS * sizeof(double) + MSE_PARTS * sizeof(double)))) {
    ga_gnet_destroy(net);
    return rc;
  }
  if ((rc = ga_gnet_set_params(net, params_host))) {
    ga_gnet_destroy(net);
    return rc;
  }
  *out = net;
  return GA_OK;
}

int ga_gnet_destroy(ga_gnet* net) {
  if (!net) return GA_OK;
  hipDeviceSynchronize();
  for (void* p : {(void*)net->params, (void*)net->m, (void*)net->v, net->wpk, (void*)net->tw,
                  (void*)net->org, (void*)net->scal, (void*)net->part, net->iw})
    if (p) hipFree(p);
  delete net;
  return GA_OK;
}

int ga_gnet_set_params(ga_gnet* net, const float* params_host) {
  if (!net) { set_error("null net"); return GA_EINVAL; }
  GA_TRY_HIP(hipDeviceSynchronize());
  if (params_host) {
    GA_TRY_HIP(hipMemcpy(net->params, params_host, GNET_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  } else {
    GA_TRY_HIP(hipMemset(net->params, 0, GNET_NPARAM * sizeof(float)));
  }
  GA_TRY_HIP(hipMemset(net->m, 0, GNET_NPARAM * sizeof(float)));
  GA_TRY_HIP(hipMemset(net->v, 0, GNET_NPARAM * sizeof(float)));
  net->adam_t = 0;
  net->packed = false;
  return GA_OK;
}

int ga_gnet_get_params(ga_gnet* net, float* params_host) {
  if (!net || !params_host) { set_error("null argument"); return GA_EINVAL; }
  GA_TRY_HIP(hipDeviceSynchronize());
  GA_TRY_HIP(hipMemcpy(params_host, net->params, GNET_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return GA_OK;
}

int ga_gnet_set_train_prec(ga_gnet* net, int prec) {
  if (!net) { set_error("null net"); return GA_EINVAL; }
  if (prec != GA_FP32 && prec != GA_BF16) { set_error("training precision must be GA_FP32 or GA_BF16"); return GA_EINVAL; }
  net->train_prec = prec;
  return GA_OK;
}

int ga_gnet_make_batch(ga_gnet* net, ga_patch* pt, const double* const* hist, const double* x,
                       int nb, int cs, const int* origins, float* in, float* tgt, void* stream) {
  if (!net || !pt || !hist || !x || !in || !tgt) { set_error("null argument"); return GA_EINVAL; }
  if (pt->dim != 3) { set_error("the learned guess needs a 3-D patch"); return GA_EINVAL; }
  for (int h = 0; h < 4; ++h)
    if (!hist[h]) { set_error("null history vector"); return GA_EINVAL; }
  int rc = check_crops(nb, cs, pt->mf, origins);
  if (rc) return rc;
  hipStream_t st = S(stream);
  if ((rc = upload_origins(net, nb, origins, st))) return rc;
  GnetFields f{{hist[0], hist[1], hist[2], hist[3]}, x};
  gnet_diff_norms(f, pt->n_free, net->part, RED_BLOCKS, st);
  launch_sum_partials(4, net->part, net->scal, st);
  gnet_make_batch(f, pt->mf, net->org, cs, nb, net->scal, in, tgt, st);
  return check_launch(0, "crop batch");
}

int ga_gnet_forward(ga_gnet* net, int nb, int cs, const int* grid3, const int* origins,
                    const float* in, float* out, void* stream) {
  if (!net || !in || !out) { set_error("null argument"); return GA_EINVAL; }
  int rc = check_crops(nb, cs, grid3, origins);
  if (rc) return rc;
  hipStream_t st = S(stream);
  TrainBufs b;
  if ((rc = upload_origins(net, nb, origins, st)) || (rc = train_bufs(net, nb, cs, &b))) return rc;
  gnet_forward_batch(net->params, in, nb, cs, grid3, net->org, b.a1, b.a2, out, b.tpk, st);
  return check_launch(0, "net forward");
}

int ga_gnet_loss_grad(ga_gnet* net, int nb, int cs, const int* grid3, const int* origins,
                      const float* in, const float* tgt, float* grad, double* loss_out,
                      void* stream) {
  if (!net || !in || !tgt || !grad) { set_error("null argument"); return GA_EINVAL; }
  int rc = check_crops(nb, cs, grid3, origins);
  if (rc) return rc;
  hipStream_t st = S(stream);
  TrainBufs b;
  if ((rc = upload_origins(net, nb, origins, st)) || (rc = train_bufs(net, nb, cs, &b))) return rc;
  gnet_forward_batch(net->params, in, nb, cs, grid3, net->org, b.a1, b.a2, b.out, b.tpk, st);
  const long long nt = (long long)nb * (cs - 6) * (cs - 6) * (cs - 6);
  double* mp = net->part + 4 * RED_BLOCKS;
  gnet_mse_grad(b.out, tgt, nt, b.d3, mp, MSE_PARTS, st);
  gnet_backward_batch(net->params, in, nb, cs, b.a1, b.a2, b.d3, b.d2, b.d1, grad, b.tpk, b.part,
                      b.wpart, st);
  if ((rc = check_launch(0, "net loss and gradient"))) return rc;
  if (loss_out) {
    std::vector<double> h(MSE_PARTS);
    GA_TRY_HIP(hipMemcpyAsync(h.data(), mp, MSE_PARTS * sizeof(double), hipMemcpyDeviceToHost, st));
    GA_TRY_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : h) s += v;
    *loss_out = s / (double)nt;
  }
  return GA_OK;
}

int ga_gnet_adam(ga_gnet* net, const float* grad, float lr, void* stream) {
  if (!net || !grad) { set_error("null argument"); return GA_EINVAL; }
  if (!(lr > 0.0f)) { set_error("lr must be positive"); return GA_EINVAL; }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  net->adam_t += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)net->adam_t));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)net->adam_t));
  gnet_adam(net->params, net->m, net->v, grad, GNET_NPARAM, lr, b1, b2, eps, c1, c2, S(stream));
  net->packed = false;
  return check_launch(0, "adam");
}

int ga_gnet_infer(ga_gnet* net, ga_patch* pt, const double* const* hist, double* x, void* stream) {
  if (!net || !pt || !hist || !x) { set_error("null argument"); return GA_EINVAL; }
  if (pt->dim != 3) { set_error("the learned guess needs a 3-D patch"); return GA_EINVAL; }
  for (int h = 0; h < 4; ++h)
    if (!hist[h]) { set_error("null history vector"); return GA_EINVAL; }
  return gnet_guess(net, pt, hist, x, S(stream));
}

}  // extern "C"
