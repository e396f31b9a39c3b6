// Batched independent patches: one order-2k step advances every patch of the
// batch together.  The patches do not interact (no interface coupling); they
// share launches instead of each paying its own:
//   - vectors are batched: patch r's free coefficients occupy entries
//     off_r .. off_r + n_r - 1 of one long vector of N = sum n_r entries, and
//     the k stage vectors are N entries apart, so the Taylor predictors and the
//     state update are single streaming launches over N;
//   - the mass and stiffness applies run as one launch per spline degree over
//     a queue of the tiles of every patch of that degree (the workgroup shape
//     depends on p, so degrees cannot share a launch);
//   - each preconditioner pass runs as one launch per register-tile class of
//     the axis length over all patches;
//   - the PCG vector updates and inner products are segment-aware: the k*R
//     systems (stage j, patch r) keep their own scalars and stop on their own.
// One PCG iteration is a fixed sequence of launches; it is captured once in a
// hipGraph (on a stream the batch owns, ordered after the caller's stream by
// events) and replayed: as many times as the previous solve of the same systems
// needed before the host first reads the per-system convergence flags, then once per
// read (the launches of an iteration skip patches whose systems have all converged,
// and a converged system's scalars stop its updates, so extra replays change
// nothing).  ga_batch_tune times the element layers per tile (ze) and
// the number of workgroups of the tile-queue launches and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ga_internal.h"
#include "kernels.h"

using namespace ga;

namespace {

struct OpGroup {
  int p = 0, mode = 0;
  std::vector<const ga_patch*> pts;
  std::vector<long long> offs;
  std::vector<int> sys;       // the patches' indices in the batch
  int ze_override = 0;        // 0: each patch's default
  int nwg = 0;                // 0: one workgroup per tile
  bool f32 = false;           // FP32 factors (mass only)
  OpGroupEntry* ents = nullptr;
  int nent = 0, total = 0;
};

struct PGroup {
  int nr = 0, pass = 0, ra = 0;
  bool f32 = false;
  PinvEntry* ents = nullptr;
  int nent = 0, nblk = 0;
};

}  // namespace

struct ga_batch {
  int R = 0, k = 1, maxit = 200;
  double rho = 0.5, tau = 0.0, rtol = 1e-10;
  double alpha[4], beta[4], gamma[4];
  std::vector<ga_patch*> pts;
  std::vector<long long> off;
  long long N = 0, maxlen = 0;
  std::vector<OpGroup> ops[2];   // mass, stiffness
  std::vector<PGroup> pgroups;
  int prec = GA_FP64;            // arithmetic of the mass solves
  std::vector<OpGroup> mass32;   // FP32 mass applies of the inner solves (GA_FP32)
  long long* seg = nullptr;      // [k*R][2]
  double *Y = nullptr, *Bv = nullptr, *X = nullptr, *work = nullptr;
  double *red = nullptr, *scal = nullptr, *host_scal = nullptr;
  hipStream_t gs = nullptr;      // stream of the captured iteration
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr, graph32 = nullptr;
  hipGraphExec_t exec = nullptr, exec32 = nullptr;
  long long n_iters = 0, n_replays = 0;
  int hint_nr = 0;               // systems of the last FP64 solve and
  std::vector<int> hint;         //   their iteration counts
  std::vector<double> taus;      // per-patch time steps (ga_batch_set_tau); empty: tau for all
};

namespace {

int upload_op_group(OpGroup& g) {
  std::vector<OpGroupEntry> h;
  int tile = 0;
  for (size_t i = 0; i < g.pts.size(); ++i) {
    const int ze = g.ze_override > 0 ? std::min(g.ze_override, g.pts[i]->n[2])
                                     : op3d_default_ze(g.mode, g.pts[i], g.f32);
    OpGroupEntry e = op3d_group_entry(g.mode, g.pts[i], ze, g.offs[i], tile, g.f32);
    e.sys = i < g.sys.size() ? g.sys[i] : 0;
    tile += e.ntiles;
    h.push_back(e);
  }
  if (g.ents) hipFree(g.ents);
  g.ents = nullptr;
  int rc = dalloc((void**)&g.ents, h.size() * sizeof(OpGroupEntry));
  if (rc) return rc;
  GA_TRY_HIP(hipMemcpy(g.ents, h.data(), h.size() * sizeof(OpGroupEntry), hipMemcpyHostToDevice));
  g.nent = (int)h.size();
  g.total = tile;
  return GA_OK;
}

int op_batch(ga_batch* b, int mode, int nr, double alpha, const double* x, double* y,
             hipStream_t st, const double* gate = nullptr) {
  for (OpGroup& g : b->ops[mode]) {
    const int cmax = op3d_max_nr(g.p, mode);
    for (int r0 = 0; r0 < nr; r0 += cmax) {
      const int c = std::min(cmax, nr - r0);
      const int nwg = g.nwg > 0 ? std::min(g.nwg, g.total) : g.total;
      if (launch_op3d_group<double>(g.p, mode, c, g.ents, g.nent, x + (size_t)r0 * b->N,
                                    y + (size_t)r0 * b->N, b->N, alpha, g.total, nwg, st,
                                    BatchGate{gate, b->R, r0}))
        return check_launch(-1, "batched operator");
    }
  }
  return GA_OK;
}

// FP32 mass applies y += M x (inner solves of the mixed-precision path)
int op_batch32(ga_batch* b, int nr, const float* x, float* y, hipStream_t st) {
  for (int r0 = 0; r0 < nr; r0 += 3) {
    const int c = std::min(3, nr - r0);
    for (OpGroup& g : b->mass32) {
      const int nwg = g.nwg > 0 ? std::min(g.nwg, g.total) : g.total;
      if (launch_op3d_group<float>(g.p, 0, c, g.ents, g.nent, x + (size_t)r0 * b->N,
                                   y + (size_t)r0 * b->N, b->N, 1.0f, g.total, nwg, st))
        return check_launch(-1, "batched FP32 mass apply");
    }
  }
  return GA_OK;
}

// entries of one preconditioner pass for nr right-hand sides, grouped by the
// register-tile class of the axis length (FP32 copies of the 1-D inverses and
// of the scaling when f32)
int build_pgroups(ga_batch* b, int nr, bool f32) {
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<PinvEntry> cls[3];
    int blk[3] = {0, 0, 0};
    for (int r = 0; r < b->R; ++r) {
      const ga_patch* pt = b->pts[r];
      const long long m0 = pt->mf[0], m1 = pt->mf[1], m2 = pt->mf[2];
      PinvEntry e{};
      e.off = b->off[r];
      e.sys = r;
      e.si = e.so = nullptr;
      long long nb = 0;
      const void* sc = f32 ? (const void*)pt->s32 : (const void*)pt->s;
      const void* A[3] = {pt->Minv[0], pt->Minv[1], pt->Minv[2]};
      if (f32)
        for (int a = 0; a < 3; ++a) A[a] = pt->Minv32[a];
      if (pass == 0) {
        e.A = A[0];
        e.L = (int)m0;
        e.si = sc;
        e.p[0] = nr * m1 * m2;
        e.p[1] = m1 * m2;
        nb = (e.p[0] + 63) / 64;
      } else if (pass == 1) {
        e.A = A[1];
        e.L = (int)m1;
        e.p[0] = m0;
        e.p[1] = m0;
        e.p[2] = m0 * m1;
        e.p[3] = m0 * m2;
        nb = (e.p[3] + 63) / 64;
      } else {
        e.A = A[2];
        e.L = (int)m2;
        e.so = sc;
        e.p[0] = m0 * m1;
        e.p[1] = m0 * m1;
        e.p[2] = 0;
        e.p[3] = m0 * m1;
        nb = (e.p[3] + 63) / 64;
      }
      const int c = pinv_ra_class(e.L);
      e.blk0 = blk[c];
      blk[c] += (int)nb;
      cls[c].push_back(e);
    }
    for (int c = 0; c < 3; ++c) {
      if (cls[c].empty()) continue;
      PGroup g;
      g.nr = nr;
      g.pass = pass;
      g.ra = c;
      g.f32 = f32;
      g.nent = (int)cls[c].size();
      g.nblk = blk[c];
      int rc = dalloc((void**)&g.ents, cls[c].size() * sizeof(PinvEntry));
      if (rc) return rc;
      GA_TRY_HIP(hipMemcpy(g.ents, cls[c].data(), cls[c].size() * sizeof(PinvEntry),
                           hipMemcpyHostToDevice));
      b->pgroups.push_back(g);
    }
  }
  return GA_OK;
}

// z = P^{-1} r for every patch (three passes, scaling folded into the first and last)
int pinv_batch(ga_batch* b, int nr, const double* r, double* z, double* t0, double* t1,
               hipStream_t st, const double* gate = nullptr) {
  const double* in[3] = {r, t1, t0};
  double* out[3] = {t1, t0, z};
  for (int pass = 0; pass < 3; ++pass)
    for (const PGroup& g : b->pgroups)
      if (g.nr == nr && g.pass == pass && !g.f32)
        launch_pinv_group<double>(pass, g.ra, g.ents, g.nent, g.nblk, nr, in[pass], out[pass], b->N, st,
                                  BatchGate{gate, b->R, 0});
  return check_launch(0, "batched preconditioner");
}

int pinv_batch32(ga_batch* b, int nr, const float* r, float* z, float* t0, float* t1,
                 hipStream_t st) {
  const float* in[3] = {r, t1, t0};
  float* out[3] = {t1, t0, z};
  for (int pass = 0; pass < 3; ++pass)
    for (const PGroup& g : b->pgroups)
      if (g.nr == nr && g.pass == pass && g.f32)
        launch_pinv_group<float>(pass, g.ra, g.ents, g.nent, g.nblk, nr, in[pass], out[pass], b->N, st);
  return check_launch(0, "batched FP32 preconditioner");
}

struct Bufs {
  double *r, *z, *p, *q, *t0, *t1;
};

Bufs bufs(ga_batch* b) {
  const size_t kn = (size_t)b->k * b->N;
  Bufs w{b->work, b->work + kn, b->work + 2 * kn, b->work + 3 * kn, b->work + 4 * kn, b->work + 5 * kn};
  return w;
}

// one PCG iteration of every active system (fixed launch sequence)
int pcg_iteration(ga_batch* b, int nr, double* x, hipStream_t st) {
  const int ns = nr * b->R;
  Bufs w = bufs(b);
  double* partA = b->red;
  launch_fill(w.q, 0.0, (size_t)nr * b->N, st);
  // the operator and preconditioner launches skip the patches whose systems have all
  // converged (device-side control: the iterations enqueued past convergence cost
  // little)
  int rc = op_batch(b, 0, nr, 1.0, w.p, w.q, st, b->scal);
  if (rc) return rc;
  launch_dot_partial_seg(ns, w.p, w.q, b->seg, partA, st);
  launch_cg_alpha(ns, partA, b->scal, st);
  launch_cg_xr_seg(ns, x, w.r, w.p, w.q, b->scal, b->seg, b->maxlen, st);
  if ((rc = pinv_batch(b, nr, w.r, w.z, w.t0, w.t1, st, b->scal))) return rc;
  launch_dot_partial_seg(ns, w.r, w.z, b->seg, partA, st);
  launch_cg_beta(ns, partA, b->scal, st);
  launch_cg_p_seg(ns, w.p, w.z, b->scal, b->seg, b->maxlen, st);
  return check_launch(0, "batched pcg iteration");
}

// buffers of the mixed-precision solve, carved from the same work area:
// the FP64 outer residual and seven FP32 vectors of k*N entries
struct Bufs32 {
  double* r64;
  float *r, *z, *p, *q, *d, *t0, *t1;
};

Bufs32 bufs32(ga_batch* b) {
  const size_t kn = (size_t)b->k * b->N;
  float* f = reinterpret_cast<float*>(b->work + kn);
  Bufs32 w{b->work, f, f + kn, f + 2 * kn, f + 3 * kn, f + 4 * kn, f + 5 * kn, f + 6 * kn};
  return w;
}

// one inner FP32 flexible-PCG iteration of every active system for M d = r
int pcg32_iteration(ga_batch* b, int nr, hipStream_t st) {
  const int ns = nr * b->R;
  Bufs32 w = bufs32(b);
  double* partA = b->red;
  double* partB = b->red + (size_t)ns * RED_BLOCKS;
  launch_fill_f32(w.q, (size_t)nr * b->N, st);
  int rc = op_batch32(b, nr, w.p, w.q, st);
  if (rc) return rc;
  launch_dot_ff(ns, w.p, w.q, b->maxlen, partA, st, b->seg);
  launch_cg_alpha(ns, partA, b->scal, st);
  launch_cg_xr_f32(ns, w.d, w.r, w.p, w.q, b->scal, b->maxlen, st, b->seg);
  if ((rc = pinv_batch32(b, nr, w.r, w.z, w.t0, w.t1, st))) return rc;
  launch_dot2_f32(ns, w.r, w.z, w.q, b->maxlen, partA, partB, st, b->seg);
  launch_cg_beta_flex(ns, partA, partB, b->scal, st);
  launch_cg_p_f32(ns, w.p, w.z, b->scal, b->maxlen, st, b->seg);
  return check_launch(0, "batched inner PCG iteration");
}

void drop_graph(ga_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->exec32) hipGraphExecDestroy(b->exec32);
  if (b->graph32) hipGraphDestroy(b->graph32);
  b->exec = b->exec32 = nullptr;
  b->graph = b->graph32 = nullptr;
}

// capture one iteration (FP64 PCG, or the FP32 inner PCG when f32) on the
// batch's stream
int capture_iteration(ga_batch* b, bool f32) {
  hipGraph_t& graph = f32 ? b->graph32 : b->graph;
  hipGraphExec_t& exec = f32 ? b->exec32 : b->exec;
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  GA_TRY_HIP(hipStreamBeginCapture(b->gs, hipStreamCaptureModeThreadLocal));
  int rc = f32 ? pcg32_iteration(b, b->k, b->gs) : pcg_iteration(b, b->k, b->X, b->gs);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->gs, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
    return GA_EDEVICE;
  }
  graph = g;
  GA_TRY_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  return GA_OK;
}

// batched PCG, zero initial guess, nr right-hand sides per patch: systems
// s = j*R + r, rhs j of patch r; x and b are [nr][N]
int solve_batch64(ga_batch* b, int nr, const double* rhs, double* x, bool graph, int* iters_out,
                  hipStream_t st) {
  const int ns = nr * b->R;
  const size_t tot = (size_t)nr * b->N;
  Bufs w = bufs(b);
  double* partA = b->red;
  launch_fill(x, 0.0, tot, st);
  launch_copy(w.r, rhs, tot, st);
  int rc = pinv_batch(b, nr, w.r, w.z, w.t0, w.t1, st);
  if (rc) return rc;
  launch_dot_partial_seg(ns, w.r, w.z, b->seg, partA, st);
  launch_cg_start(ns, partA, nullptr, b->scal, b->rtol * b->rtol, st);
  launch_copy(w.p, w.z, tot, st);
  if (check_launch(0, "batched pcg start")) return GA_EDEVICE;
  const bool use_graph = graph && nr == b->k && x == b->X;
  if (use_graph && !b->exec && (rc = capture_iteration(b, false))) return rc;
  // iterations run before the first read of the convergence flags: as many as the
  // previous solve of ns systems needed (an iteration leaves a converged system
  // unchanged and its launches skip it, so no iterate depends on this)
  int ahead = 0;
  if (b->hint_nr == ns) {
    for (int s = 0; s < ns; ++s) ahead = std::max(ahead, b->hint[s]);
    ahead = std::min(ahead, b->maxit);
  }
  for (int it = 0;; ++it) {
    if (it >= ahead) {
      GA_TRY_HIP(hipMemcpyAsync(b->host_scal, b->scal, sizeof(double) * NSCAL * ns,
                                hipMemcpyDeviceToHost, st));
      GA_TRY_HIP(hipStreamSynchronize(st));
      bool any = false;
      for (int s = 0; s < ns; ++s) any |= b->host_scal[s * NSCAL + S_ACTIVE] != 0.0;
      if (!any || it >= b->maxit) break;
    }
    if (use_graph) {
      GA_TRY_HIP(hipGraphLaunch(b->exec, st));
      b->n_replays += 1;
    } else if ((rc = pcg_iteration(b, nr, x, st))) {
      return rc;
    }
    b->n_iters += 1;
  }
  bool ok = true;
  b->hint_nr = ns;
  b->hint.assign(ns, 0);
  for (int s = 0; s < ns; ++s) {
    const double* sc = b->host_scal + s * NSCAL;
    if (iters_out) iters_out[s] = (int)sc[S_ITERS];
    b->hint[s] = (int)sc[S_ITERS];
    if (sc[S_ACTIVE] != 0.0 || !std::isfinite(sc[S_RZ])) ok = false;
  }
  if (!ok) {
    set_error("batched PCG did not converge within maxit");
    return GA_ENOCONV;
  }
  return GA_OK;
}

int read_batch_scalars(ga_batch* b, int ns, hipStream_t st) {
  GA_TRY_HIP(hipMemcpyAsync(b->host_scal, b->scal, sizeof(double) * NSCAL * ns,
                            hipMemcpyDeviceToHost, st));
  GA_TRY_HIP(hipStreamSynchronize(st));
  return GA_OK;
}

// Batched mixed-precision solve, zero initial guess: FP64 iterative refinement
// (outer residual r = b - M x with the FP64 factors, stop when
// sqrt(r^T P^{-1} r) <= rtol sqrt(b^T P^{-1} b) per system, dots in FP64) around
// FP32 flexible PCG corrections M d = r that reduce their residual by 1e-4.  A
// system that has met its tolerance gets a zero correction (its inner residual
// is cleared) while the others go on.  x and rhs are [nr][N] in FP64.
int solve_batch_mixed(ga_batch* b, int nr, const double* rhs, double* x, bool graph,
                      int* iters_out, hipStream_t st) {
  const int ns = nr * b->R;
  const size_t tot = (size_t)nr * b->N;
  Bufs32 w = bufs32(b);
  double* partA = b->red;
  double* partB = b->red + (size_t)ns * RED_BLOCKS;
  const double inner_tol = 1e-4;
  const bool use_graph = graph && nr == b->k;
  int rc;
  if (use_graph && !b->exec32 && (rc = capture_iteration(b, true))) return rc;
  launch_fill(x, 0.0, tot, st);
  launch_to_f32(w.r, rhs, tot, st);
  if ((rc = pinv_batch32(b, nr, w.r, w.z, w.t0, w.t1, st))) return rc;
  launch_dot_df(ns, rhs, w.z, b->maxlen, partB, st, b->seg);
  launch_sum_partials(ns, partB, b->scal, st);
  if ((rc = read_batch_scalars(b, ns, st))) return rc;
  std::vector<double> bn2(ns), rz(ns);
  std::vector<int> inner(ns, 0);
  for (int s = 0; s < ns; ++s) rz[s] = bn2[s] = b->host_scal[s];
  auto seg_of = [&](int s, size_t& off, size_t& len) {
    const int j = s / b->R, r = s % b->R;
    off = (size_t)j * b->N + (size_t)b->off[r];
    len = (size_t)b->pts[r]->n_free;
  };
  bool conv = false;
  for (int outer = 0; outer < 50; ++outer) {
    if (outer > 0) {   // preconditioned outer residual
      launch_to_f32(w.r, w.r64, tot, st);
      if ((rc = pinv_batch32(b, nr, w.r, w.z, w.t0, w.t1, st))) return rc;
      launch_dot_df(ns, w.r64, w.z, b->maxlen, partA, st, b->seg);
      launch_sum_partials(ns, partA, b->scal, st);
      if ((rc = read_batch_scalars(b, ns, st))) return rc;
      for (int s = 0; s < ns; ++s) rz[s] = b->host_scal[s];
    }
    bool all = true;
    for (int s = 0; s < ns; ++s) {
      const bool done = !(bn2[s] > 0.0) || rz[s] <= b->rtol * b->rtol * bn2[s];
      if (!done) {
        all = false;
      } else {   // no correction for a converged system
        size_t off, len;
        seg_of(s, off, len);
        launch_fill_f32(w.r + off, len, st);
        launch_fill_f32(w.z + off, len, st);
      }
    }
    int used = 0;
    for (int s = 0; s < ns; ++s) used = std::max(used, inner[s]);
    if (all) { conv = true; break; }
    if (used >= b->maxit) break;
    launch_fill_f32(w.d, tot, st);
    launch_dot_ff(ns, w.r, w.z, b->maxlen, partA, st, b->seg);
    launch_cg_start(ns, partA, nullptr, b->scal, inner_tol * inner_tol, st);
    launch_copy_f32(w.p, w.z, tot, st);
    if (check_launch(0, "batched inner PCG start")) return GA_EDEVICE;
    for (int it = 0; it < 20; ++it) {
      if ((rc = read_batch_scalars(b, ns, st))) return rc;
      bool any = false;
      for (int s = 0; s < ns; ++s) any |= b->host_scal[s * NSCAL + S_ACTIVE] != 0.0;
      if (!any) break;
      if (use_graph) {
        GA_TRY_HIP(hipGraphLaunch(b->exec32, st));
        b->n_replays += 1;
      } else if ((rc = pcg32_iteration(b, nr, st))) {
        return rc;
      }
      b->n_iters += 1;
    }
    if ((rc = read_batch_scalars(b, ns, st))) return rc;
    for (int s = 0; s < ns; ++s) inner[s] += (int)b->host_scal[s * NSCAL + S_ITERS];
    // x += d; r = b - M x in FP64
    launch_add_f32(x, w.d, tot, st);
    launch_copy(w.r64, rhs, tot, st);
    if ((rc = op_batch(b, 0, nr, -1.0, x, w.r64, st))) return rc;
  }
  for (int s = 0; s < ns; ++s) {
    if (iters_out) iters_out[s] = inner[s];
    if (!std::isfinite(rz[s])) conv = false;
  }
  if (!conv) {
    set_error("batched mixed-precision solve did not converge within maxit");
    return GA_ENOCONV;
  }
  return GA_OK;
}

int solve_batch(ga_batch* b, int nr, const double* rhs, double* x, bool graph, int* iters_out,
                hipStream_t st) {
  if (b->prec == GA_FP32) return solve_batch_mixed(b, nr, rhs, x, graph, iters_out, st);
  return solve_batch64(b, nr, rhs, x, graph, iters_out, st);
}

void free_batch(ga_batch* b) {
  drop_graph(b);
  for (int m = 0; m < 2; ++m)
    for (OpGroup& g : b->ops[m])
      if (g.ents) hipFree(g.ents);
  for (OpGroup& g : b->mass32)
    if (g.ents) hipFree(g.ents);
  for (PGroup& g : b->pgroups)
    if (g.ents) hipFree(g.ents);
  for (void* p : {(void*)b->seg, (void*)b->Y, (void*)b->Bv, (void*)b->X, (void*)b->work,
                  (void*)b->red, (void*)b->scal})
    if (p) hipFree(p);
  if (b->host_scal) hipHostFree(b->host_scal);
  for (hipEvent_t e : b->ev)
    if (e) hipEventDestroy(e);
  if (b->gs) hipStreamDestroy(b->gs);
  delete b;
}

// order the batch stream after the caller's stream (or the reverse)
int join(hipStream_t from, hipStream_t to, hipEvent_t ev) {
  GA_TRY_HIP(hipEventRecord(ev, from));
  GA_TRY_HIP(hipStreamWaitEvent(to, ev, 0));
  return GA_OK;
}

}  // namespace

extern "C" {

int ga_batch_create(int npatch, ga_patch* const* patches, int k, double rho, double tau,
                    double rtol, int maxit, ga_batch** out) {
  if (!out || !patches) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  if (npatch < 1 || npatch > 64) { set_error("npatch must be in 1..64"); return GA_EINVAL; }
  if (k < 1 || k > 4) { set_error("k must be in 1..4"); return GA_EINVAL; }
  if (!(rho >= 0.0 && rho < 1.0) || !(tau > 0.0) || !(rtol > 0.0) || maxit < 1) {
    set_error("bad rho/tau/rtol/maxit");
    return GA_EINVAL;
  }
  for (int r = 0; r < npatch; ++r) {
    const ga_patch* pt = patches[r];
    if (!pt) { set_error("null patch"); return GA_EINVAL; }
    if (pt->dim != 3 || pt->p < 2 || pt->p > 4) {
      set_error("batched patches must be 3-D with p in 2..4");
      return GA_EINVAL;
    }
    for (int a = 0; a < 3; ++a)
      if (!pinv_axis_supported(pt->mf[a])) {
        set_error("batched patches need at most 256 free coefficients per axis");
        return GA_EINVAL;
      }
  }
  ga_batch* b = new ga_batch();
  b->R = npatch;
  b->k = k;
  b->rho = rho;
  b->tau = tau;
  b->rtol = rtol;
  b->maxit = maxit;
  for (int j = 0; j < k; ++j) {
    if (j < k - 1) block_j_params(rho, b->alpha[j], b->beta[j], b->gamma[j]);
    else block_k_params(rho, b->alpha[j], b->beta[j], b->gamma[j]);
  }
  for (int r = 0; r < npatch; ++r) {
    b->pts.push_back(patches[r]);
    b->off.push_back(b->N);
    b->N += patches[r]->n_free;
    b->maxlen = std::max(b->maxlen, patches[r]->n_free);
  }
  int rc = GA_OK;
  auto fail = [&](int code) {
    free_batch(b);
    return code;
  };
  for (int mode = 0; mode < 2; ++mode)
    for (int p = 2; p <= 4; ++p) {
      OpGroup g;
      g.p = p;
      g.mode = mode;
      for (int r = 0; r < npatch; ++r)
        if (patches[r]->p == p) {
          g.pts.push_back(patches[r]);
          g.offs.push_back(b->off[r]);
          g.sys.push_back(r);
        }
      if (g.pts.empty()) continue;
      b->ops[mode].push_back(g);
      if ((rc = upload_op_group(b->ops[mode].back()))) return fail(rc);
    }
  if ((rc = build_pgroups(b, 1, false))) return fail(rc);
  if (k > 1 && (rc = build_pgroups(b, k, false))) return fail(rc);
  std::vector<long long> seg;
  for (int j = 0; j < k; ++j)
    for (int r = 0; r < npatch; ++r) {
      seg.push_back((long long)j * b->N + b->off[r]);
      seg.push_back(patches[r]->n_free);
    }
  const size_t kn = (size_t)k * b->N;
  const int ns = k * npatch;
  if ((rc = dalloc((void**)&b->seg, seg.size() * sizeof(long long))) ||
      (rc = dalloc((void**)&b->Y, kn * 8)) || (rc = dalloc((void**)&b->Bv, kn * 8)) ||
      (rc = dalloc((void**)&b->X, kn * 8)) || (rc = dalloc((void**)&b->work, 6 * kn * 8)) ||
      (rc = dalloc((void**)&b->red, (size_t)2 * ns * RED_BLOCKS * 8)) ||
      (rc = dalloc((void**)&b->scal, (size_t)ns * NSCAL * 8)))
    return fail(rc);
  if (hipHostMalloc((void**)&b->host_scal, (size_t)ns * NSCAL * 8, hipHostMallocDefault) != hipSuccess) {
    set_error("pinned host allocation failed");
    return fail(GA_ENOMEM);
  }
  if (hipMemcpy(b->seg, seg.data(), seg.size() * sizeof(long long), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipStreamCreateWithFlags(&b->gs, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming) != hipSuccess) {
    set_error("batch stream/event setup failed");
    return fail(GA_EDEVICE);
  }
  *out = b;
  return GA_OK;
}

int ga_batch_set_precision(ga_batch* b, int prec, void* stream) {
  if (!b) { set_error("null batch"); return GA_EINVAL; }
  if (prec != GA_FP64 && prec != GA_FP32) { set_error("prec must be GA_FP64 or GA_FP32"); return GA_EINVAL; }
  drop_graph(b);
  b->prec = prec;
  if (prec == GA_FP64 || !b->mass32.empty()) return GA_OK;
  hipStream_t st = S(stream);
  int rc;
  for (ga_patch* pt : b->pts)
    if ((rc = mixed_setup(pt, st))) return rc;
  for (const OpGroup& g64 : b->ops[0]) {
    OpGroup g;
    g.p = g64.p;
    g.mode = 0;
    g.pts = g64.pts;
    g.offs = g64.offs;
    g.sys = g64.sys;
    g.ze_override = g64.ze_override;
    g.nwg = g64.nwg;
    g.f32 = true;
    b->mass32.push_back(g);
    if ((rc = upload_op_group(b->mass32.back()))) return rc;
  }
  if ((rc = build_pgroups(b, 1, true))) return rc;
  if (b->k > 1 && (rc = build_pgroups(b, b->k, true))) return rc;
  GA_TRY_HIP(hipStreamSynchronize(st));
  return check_launch(0, "batched mixed-precision setup");
}

int ga_batch_set_tau(ga_batch* b, const double* tau_host) {
  if (!b) { set_error("null batch"); return GA_EINVAL; }
  if (!tau_host) { b->taus.clear(); return GA_OK; }
  for (int r = 0; r < b->R; ++r)
    if (!(tau_host[r] > 0.0) || !std::isfinite(tau_host[r])) {
      set_error("time steps must be positive and finite");
      return GA_EINVAL;
    }
  b->taus.assign(tau_host, tau_host + b->R);
  return GA_OK;
}

int ga_batch_destroy(ga_batch* b) {
  if (!b) return GA_OK;
  hipDeviceSynchronize();
  free_batch(b);
  return GA_OK;
}

int ga_batch_info(const ga_batch* b, long long* n_total, long long* offsets, long long* replays) {
  if (!b) { set_error("null batch"); return GA_EINVAL; }
  if (n_total) *n_total = b->N;
  if (offsets)
    for (int r = 0; r < b->R; ++r) offsets[r] = b->off[r];
  if (replays) *replays = b->n_replays;
  return GA_OK;
}

int ga_batch_tune(ga_batch* b, int reps, double* best_ms, void* stream) {
  if (!b || reps < 1) { set_error("bad argument"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  Bufs w = bufs(b);
  hipEvent_t e0, e1;
  GA_TRY_HIP(hipEventCreate(&e0));
  GA_TRY_HIP(hipEventCreate(&e1));
  double total = 0.0;
  int rc = GA_OK;
  const int nr = std::min(b->k, 3);
  launch_fill(w.t0, 0.0, (size_t)b->k * b->N, st);
  launch_fill(w.t1, 0.0, (size_t)b->k * b->N, st);
  float* t32 = reinterpret_cast<float*>(w.t0);
  for (int mode = 0; mode < 3 && !rc; ++mode)
    for (OpGroup& g : mode < 2 ? b->ops[mode] : b->mass32) {
      int best_ze = g.ze_override, best_nwg = g.nwg;
      double best = 1e30;
      std::vector<int> zes = {0, 2, 4, 8, 16, 32};
      for (int ze : zes) {
        g.ze_override = ze;
        if ((rc = upload_op_group(g))) break;
        for (int nwgc : {0, 2048, 1024}) {
          if (nwgc > 0 && nwgc >= g.total) continue;
          g.nwg = nwgc;
          const int nwg = nwgc > 0 ? nwgc : g.total;
          // warm-up, then timed launches (k right-hand sides, scratch vectors)
          const int nrg = std::min(nr, op3d_max_nr(g.p, g.mode));
          auto launch = [&]() {
            if (g.f32)
              launch_op3d_group<float>(g.p, 0, nrg, g.ents, g.nent, t32, t32 + (size_t)nrg * b->N,
                                       b->N, 1.0f, g.total, nwg, st);
            else
              launch_op3d_group<double>(g.p, g.mode, nrg, g.ents, g.nent, w.t0, w.t1, b->N, 1.0,
                                        g.total, nwg, st);
          };
          launch();
          hipEventRecord(e0, st);
          for (int i = 0; i < reps; ++i) launch();
          hipEventRecord(e1, st);
          if (hipEventSynchronize(e1) != hipSuccess) { rc = check_launch(-1, "tuning"); break; }
          float ms = 0.f;
          hipEventElapsedTime(&ms, e0, e1);
          if (ms < best) { best = ms; best_ze = ze; best_nwg = nwgc; }
        }
        if (rc) break;
      }
      if (rc) break;
      g.ze_override = best_ze;
      g.nwg = best_nwg;
      if ((rc = upload_op_group(g))) break;
      total += best / reps;
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  drop_graph(b);   // the captured iteration used the old launch shapes
  if (best_ms) *best_ms = total;
  return check_launch(0, "tuning");
}

int ga_batch_init_state(ga_batch* b, const double* U0, const double* V0, double* const* state,
                        void* stream) {
  if (!b || !U0 || !V0 || !state) { set_error("null argument"); return GA_EINVAL; }
  for (int s = 0; s < 3 * b->k; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = b->N;
  launch_copy(state[0], U0, n, st);
  launch_copy(state[1], V0, n, st);
  for (int a = 0; a <= 3 * b->k - 3; ++a) {
    launch_fill(b->Y, 0.0, n, st);
    int rc = op_batch(b, 1, 1, -1.0, state[a], b->Y, st);
    if (rc) return rc;
    if ((rc = solve_batch(b, 1, b->Y, state[a + 2], false, nullptr, st))) return rc;
  }
  return GA_OK;
}

int ga_batch_step(ga_batch* b, double* const* state, int nsteps, int use_graph, int* iters_out,
                  void* stream) {
  if (!b || !state || nsteps < 0) { set_error("bad argument"); return GA_EINVAL; }
  const int k = b->k, ns = 3 * k;
  for (int s = 0; s < ns; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t cst = S(stream);
  hipStream_t st = use_graph ? b->gs : cst;
  int rc;
  if (use_graph && (rc = join(cst, st, b->ev[0]))) return rc;
  const size_t n = b->N;
  StatePtrs sp;
  for (int s = 0; s < 12; ++s) sp.L[s] = s < ns ? state[s] : nullptr;
  Coefs cf;
  for (int j = 0; j < 4; ++j) {
    cf.alpha[j] = j < k ? b->alpha[j] : 1.0;
    cf.beta[j] = j < k ? b->beta[j] : 0.0;
    cf.gamma[j] = j < k ? b->gamma[j] : 0.0;
  }
  std::vector<int> its((size_t)k * b->R);
  // one patch's segment of the batched state (per-patch time steps)
  auto seg_ptrs = [&](int r) {
    StatePtrs q;
    for (int s = 0; s < 12; ++s) q.L[s] = s < ns ? state[s] + b->off[r] : nullptr;
    return q;
  };
  for (int step = 0; step < nsteps; ++step) {
    if (b->taus.empty()) {
      launch_predict(k, b->tau, sp, b->Y, n, st);
    } else {
      for (int r = 0; r < b->R; ++r)
        launch_predict_seg(k, b->taus[r], seg_ptrs(r), b->Y + b->off[r], b->pts[r]->n_free, n, st);
    }
    launch_fill(b->Bv, 0.0, (size_t)k * n, st);
    if ((rc = op_batch(b, 1, k, -1.0, b->Y, b->Bv, st))) return rc;
    if ((rc = solve_batch(b, k, b->Bv, b->X, use_graph != 0, its.data(), st))) return rc;
    if (iters_out)
      for (size_t s = 0; s < its.size(); ++s) iters_out[(size_t)step * its.size() + s] = its[s];
    if (b->taus.empty()) {
      launch_update(k, b->tau, cf, sp, b->X, n, st);
    } else {
      for (int r = 0; r < b->R; ++r)
        launch_update_seg(k, b->taus[r], cf, seg_ptrs(r), b->X + b->off[r], b->pts[r]->n_free, n, st);
    }
    if (check_launch(0, "batched update")) return GA_EDEVICE;
  }
  if (use_graph && (rc = join(st, cst, b->ev[1]))) return rc;
  GA_TRY_HIP(hipStreamSynchronize(cst));
  return GA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Glued (C^0) multi-patch domain (Sec. 5.3) with the additive Schwarz mass
// preconditioner (Sec. 5.5): a brick of P_x x P_y x P_z patches, each n elements
// and degree p.  The patch work runs through a batch over the patches' local
// free coefficients (interface faces free, outer faces Dirichlet); the PCG and
// the time stepping run on the global unknowns:
//   Op x = sum_r G^(r)T Op^(r) G^(r) x          (gather, batched applies, scatter-add)
//   P_ad^{-1} r = sum_r R^(r)T (P^(r))^{-1} R^(r) r
// with G^(r) = R^(r) the map from patch r's free coefficients to global indices.

struct ga_mp {
  int P[3] = {1, 1, 1}, n = 0, p = 0, k = 1, maxit = 200;
  double tau = 0.0, rtol = 1e-10;
  double alpha[4], beta[4], gamma[4];
  std::vector<ga_patch*> pts;      // owned
  ga_batch* b = nullptr;           // owned
  long long Ng = 0, Nl = 0;
  int mfg[3] = {1, 1, 1};
  int* map = nullptr;              // [Nl] local free index -> global unknown
  double *Y = nullptr, *Bv = nullptr, *X = nullptr, *gw = nullptr;  // global vectors
  double *red = nullptr, *scal = nullptr, *host_scal = nullptr;
  int hint_nr = 0;                 // systems of the last solve and
  std::vector<int> hint;           //   their iteration counts
};

namespace {

// y += alpha Op x on global vectors (mode 0 mass, 1 stiffness), nr right-hand sides
int mp_op(ga_mp* m, int mode, int nr, double alpha, const double* x, double* y, hipStream_t st) {
  Bufs w = bufs(m->b);
  launch_gather(nr, x, m->Ng, m->map, m->Nl, w.r, st);
  launch_fill(w.z, 0.0, (size_t)nr * m->Nl, st);
  int rc = op_batch(m->b, mode, nr, 1.0, w.r, w.z, st);
  if (rc) return rc;
  launch_scatter_add(nr, w.z, m->Nl, m->map, alpha, y, m->Ng, st);
  return check_launch(0, "multi-patch operator");
}

// z = P_ad^{-1} r
int mp_pinv(ga_mp* m, int nr, const double* r, double* z, hipStream_t st) {
  Bufs w = bufs(m->b);
  launch_gather(nr, r, m->Ng, m->map, m->Nl, w.r, st);
  int rc = pinv_batch(m->b, nr, w.r, w.z, w.t0, w.t1, st);
  if (rc) return rc;
  launch_fill(z, 0.0, (size_t)nr * m->Ng, st);
  launch_scatter_add(nr, w.z, m->Nl, m->map, 1.0, z, m->Ng, st);
  return check_launch(0, "additive Schwarz preconditioner");
}

// PCG with P_ad for nr systems of Ng unknowns, zero initial guess (stopping rule as
// for one patch: preconditioned residual relative to that of b)
int mp_solve(ga_mp* m, int nr, const double* rhs, double* x, int* iters_out, hipStream_t st) {
  const size_t n = m->Ng, tot = (size_t)nr * n;
  double* r = m->gw;
  double* z = r + (size_t)m->k * n;
  double* pv = z + (size_t)m->k * n;
  double* q = pv + (size_t)m->k * n;
  launch_fill(x, 0.0, tot, st);
  launch_copy(r, rhs, tot, st);
  int rc = mp_pinv(m, nr, r, z, st);
  if (rc) return rc;
  launch_dot_partial(nr, r, z, n, m->red, st);
  launch_cg_start(nr, m->red, nullptr, m->scal, m->rtol * m->rtol, st);
  launch_copy(pv, z, tot, st);
  // iterations enqueued before the first read of the convergence flags: one
  // fewer than the fewest the previous solve of nr systems needed.  An
  // iteration leaves a converged system unchanged (zero step, no new
  // direction), so this changes no iterate, only when the host looks.
  int ahead = 0;
  if (m->hint_nr == nr) {
    ahead = m->maxit;
    for (int s = 0; s < nr; ++s) ahead = std::min(ahead, m->hint[s] - 1);
    ahead = std::max(ahead, 0);
  }
  for (int it = 0;; ++it) {
    if (it >= ahead) {
      GA_TRY_HIP(hipMemcpyAsync(m->host_scal, m->scal, sizeof(double) * NSCAL * nr,
                                hipMemcpyDeviceToHost, st));
      GA_TRY_HIP(hipStreamSynchronize(st));
      bool any = false;
      for (int s = 0; s < nr; ++s) any |= m->host_scal[s * NSCAL + S_ACTIVE] != 0.0;
      if (!any || it >= m->maxit) break;
    }
    launch_fill(q, 0.0, tot, st);
    if ((rc = mp_op(m, 0, nr, 1.0, pv, q, st))) return rc;
    launch_dot_partial(nr, pv, q, n, m->red, st);
    launch_cg_alpha(nr, m->red, m->scal, st);
    launch_cg_xr(nr, x, r, pv, q, m->scal, n, st);
    if ((rc = mp_pinv(m, nr, r, z, st))) return rc;
    launch_dot_partial(nr, r, z, n, m->red, st);
    launch_cg_beta(nr, m->red, m->scal, st);
    launch_cg_p(nr, pv, z, m->scal, n, st);
    if (check_launch(0, "multi-patch pcg")) return GA_EDEVICE;
  }
  bool ok = true;
  m->hint_nr = nr;
  m->hint.assign(nr, 0);
  for (int s = 0; s < nr; ++s) {
    const double* sc = m->host_scal + s * NSCAL;
    if (iters_out) iters_out[s] = (int)sc[S_ITERS];
    m->hint[s] = (int)sc[S_ITERS];
    if (sc[S_ACTIVE] != 0.0 || !std::isfinite(sc[S_RZ])) ok = false;
  }
  if (!ok) { set_error("multi-patch PCG did not converge within maxit"); return GA_ENOCONV; }
  return GA_OK;
}

void free_mp(ga_mp* m) {
  if (m->b) ga_batch_destroy(m->b);
  for (ga_patch* pt : m->pts)
    if (pt) ga_destroy_patch(pt);
  for (void* q : {(void*)m->map, (void*)m->Y, (void*)m->Bv, (void*)m->X, (void*)m->gw,
                  (void*)m->red, (void*)m->scal})
    if (q) hipFree(q);
  if (m->host_scal) hipHostFree(m->host_scal);
  delete m;
}

}  // namespace

extern "C" {

int ga_mp_create(const int* P, int n_el, int p, const double* const* ctrl_host, int k, double rho,
                 double tau, double rtol, int maxit, void* stream, ga_mp** out) {
  if (!P || !ctrl_host || !out) { set_error("null argument"); return GA_EINVAL; }
  *out = nullptr;
  const int R = P[0] * P[1] * P[2];
  if (P[0] < 1 || P[1] < 1 || P[2] < 1 || R > 64) { set_error("brick must have 1..64 patches"); return GA_EINVAL; }
  if (p < 2 || p > 4 || n_el < 1) { set_error("need p in 2..4 and n_el >= 1"); return GA_EINVAL; }
  if (k < 1 || k > 4 || !(tau > 0.0) || !(rtol > 0.0) || maxit < 1 || !(rho >= 0.0 && rho < 1.0)) {
    set_error("bad k/rho/tau/rtol/maxit");
    return GA_EINVAL;
  }
  for (int r = 0; r < R; ++r)
    if (!ctrl_host[r]) { set_error("null control points"); return GA_EINVAL; }
  ga_mp* m = new ga_mp();
  for (int a = 0; a < 3; ++a) m->P[a] = P[a];
  m->n = n_el;
  m->p = p;
  m->k = k;
  m->tau = tau;
  m->rtol = rtol;
  m->maxit = maxit;
  for (int j = 0; j < k; ++j) {
    if (j < k - 1) block_j_params(rho, m->alpha[j], m->beta[j], m->gamma[j]);
    else block_k_params(rho, m->alpha[j], m->beta[j], m->gamma[j]);
  }
  const int mm = n_el + p;                       // coefficients per patch and axis
  long long Ng = 1;
  for (int a = 0; a < 3; ++a) {
    m->mfg[a] = P[a] * (mm - 1) - 1;             // global unknowns per axis
    Ng *= m->mfg[a];
  }
  m->Ng = Ng;
  int rc = GA_OK;
  std::vector<int> map;
  const int nn[3] = {n_el, n_el, n_el};
  for (int r = 0; r < R; ++r) {
    const int b[3] = {r % P[0], (r / P[0]) % P[1], r / (P[0] * P[1])};
    unsigned faces = 0;
    for (int a = 0; a < 3; ++a) {
      if (b[a] == 0) faces |= 1u << (2 * a);
      if (b[a] == P[a] - 1) faces |= 1u << (2 * a + 1);
    }
    ga_patch* pt = nullptr;
    if ((rc = ga_setup_patch_ex(3, nn, p, ctrl_host[r], faces, stream, &pt))) { free_mp(m); return rc; }
    m->pts.push_back(pt);
    // G^(r): local free (co-lex) -> global unknown: g_a = b_a (m-1) + i_a - 1
    for (int iz = 0; iz < pt->mf[2]; ++iz)
      for (int iy = 0; iy < pt->mf[1]; ++iy)
        for (int ix = 0; ix < pt->mf[0]; ++ix) {
          const long long gx = (long long)b[0] * (mm - 1) + pt->lo[0] + ix - 1;
          const long long gy = (long long)b[1] * (mm - 1) + pt->lo[1] + iy - 1;
          const long long gz = (long long)b[2] * (mm - 1) + pt->lo[2] + iz - 1;
          map.push_back((int)(gx + (long long)m->mfg[0] * (gy + (long long)m->mfg[1] * gz)));
        }
  }
  if (Ng > (1LL << 31) - 1) { set_error("too many unknowns"); free_mp(m); return GA_EINVAL; }
  m->Nl = (long long)map.size();
  if ((rc = ga_batch_create(R, m->pts.data(), k, rho, tau, rtol, maxit, &m->b))) { free_mp(m); return rc; }
  const size_t kn = (size_t)k * Ng;
  if ((rc = dalloc((void**)&m->map, map.size() * sizeof(int))) || (rc = dalloc((void**)&m->Y, kn * 8)) ||
      (rc = dalloc((void**)&m->Bv, kn * 8)) || (rc = dalloc((void**)&m->X, kn * 8)) ||
      (rc = dalloc((void**)&m->gw, 4 * kn * 8)) ||
      (rc = dalloc((void**)&m->red, (size_t)k * RED_BLOCKS * 8)) ||
      (rc = dalloc((void**)&m->scal, (size_t)k * NSCAL * 8))) {
    free_mp(m);
    return rc;
  }
  if (hipHostMalloc((void**)&m->host_scal, (size_t)k * NSCAL * 8, hipHostMallocDefault) != hipSuccess) {
    set_error("pinned host allocation failed");
    free_mp(m);
    return GA_ENOMEM;
  }
  if (hipMemcpy(m->map, map.data(), map.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("map upload failed");
    free_mp(m);
    return GA_EDEVICE;
  }
  *out = m;
  return GA_OK;
}

int ga_mp_destroy(ga_mp* m) {
  if (!m) return GA_OK;
  hipDeviceSynchronize();
  free_mp(m);
  return GA_OK;
}

int ga_mp_info(const ga_mp* m, long long* n_global, int* mfg, long long* n_local) {
  if (!m) { set_error("null multi-patch domain"); return GA_EINVAL; }
  if (n_global) *n_global = m->Ng;
  if (mfg) for (int a = 0; a < 3; ++a) mfg[a] = m->mfg[a];
  if (n_local) *n_local = m->Nl;
  return GA_OK;
}

int ga_mp_apply(ga_mp* m, char which, int nrhs, const double* x, double* y, void* stream) {
  if (!m || !x || !y) { set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1 || nrhs > m->k) { set_error("nrhs must be in 1..k"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  if (which == 'P') return mp_pinv(m, nrhs, x, y, st);
  if (which != 'M' && which != 'K') { set_error("which must be 'M', 'K' or 'P'"); return GA_EINVAL; }
  launch_fill(y, 0.0, (size_t)nrhs * m->Ng, st);
  return mp_op(m, which == 'K' ? 1 : 0, nrhs, 1.0, x, y, st);
}

int ga_mp_mass_solve(ga_mp* m, int nrhs, const double* rhs, double* x, int* iters_out,
                     void* stream) {
  if (!m || !rhs || !x) { set_error("null argument"); return GA_EINVAL; }
  if (nrhs < 1 || nrhs > m->k) { set_error("nrhs must be in 1..k"); return GA_EINVAL; }
  return mp_solve(m, nrhs, rhs, x, iters_out, S(stream));
}

int ga_mp_init_state(ga_mp* m, const double* U0, const double* V0, double* const* state,
                     void* stream) {
  if (!m || !U0 || !V0 || !state) { set_error("null argument"); return GA_EINVAL; }
  for (int s = 0; s < 3 * m->k; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = m->Ng;
  launch_copy(state[0], U0, n, st);
  launch_copy(state[1], V0, n, st);
  for (int a = 0; a <= 3 * m->k - 3; ++a) {
    launch_fill(m->Bv, 0.0, n, st);
    int rc = mp_op(m, 1, 1, -1.0, state[a], m->Bv, st);
    if (rc) return rc;
    if ((rc = mp_solve(m, 1, m->Bv, state[a + 2], nullptr, st))) return rc;
  }
  return GA_OK;
}

int ga_mp_step(ga_mp* m, double* const* state, int nsteps, int* iters_out, void* stream) {
  if (!m || !state || nsteps < 0) { set_error("bad argument"); return GA_EINVAL; }
  const int k = m->k, ns = 3 * k;
  for (int s = 0; s < ns; ++s)
    if (!state[s]) { set_error("null state vector"); return GA_EINVAL; }
  hipStream_t st = S(stream);
  const size_t n = m->Ng;
  StatePtrs sp;
  for (int s = 0; s < 12; ++s) sp.L[s] = s < ns ? state[s] : nullptr;
  Coefs cf;
  for (int j = 0; j < 4; ++j) {
    cf.alpha[j] = j < k ? m->alpha[j] : 1.0;
    cf.beta[j] = j < k ? m->beta[j] : 0.0;
    cf.gamma[j] = j < k ? m->gamma[j] : 0.0;
  }
  int its[4];
  for (int step = 0; step < nsteps; ++step) {
    launch_predict(k, m->tau, sp, m->Y, n, st);
    launch_fill(m->Bv, 0.0, (size_t)k * n, st);
    int rc = mp_op(m, 1, k, -1.0, m->Y, m->Bv, st);
    if (rc) return rc;
    if ((rc = mp_solve(m, k, m->Bv, m->X, its, st))) return rc;
    if (iters_out)
      for (int j = 0; j < k; ++j) iters_out[(size_t)step * k + j] = its[j];
    launch_update(k, m->tau, cf, sp, m->X, n, st);
    if (check_launch(0, "multi-patch update")) return GA_EDEVICE;
  }
  GA_TRY_HIP(hipStreamSynchronize(st));
  return GA_OK;
}

}  // extern "C"
