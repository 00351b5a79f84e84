// Host runtime of libnnc: contexts, network registry and the three oracle
// calls of the reduced-space formulation (Section 3.2 of arXiv 2509.22462):
// eval_g (Eq. 5), eval_jac_g, eval_hess_lag (Section 3.2.1, Eq. 6).
//
// Data layout in HBM (all buffers allocated at nnc_net_create):
//   * weights per layer in the compute type, W_l [d_l'][d_{l-1}'] and a
//     transposed copy W_l^T [d_{l-1}'][d_l'] (d' = width padded to 64, the
//     input width to 64), so that every GEMM of both sweeps is K-contiguous;
//     the output layer also in FP64 (W_L and W_L^T) for the FP64 residual and
//     the FP64 lambda-weighted adjoint;
//   * per point and layer: z_l (FP64), a_l, sigma'_l, zbar_l and s_l;
//   * tangents stored "transposed", one row per tangent column (b, j):
//     [B*n][d_l'] so that rows are feature-contiguous; G_l of the reverse
//     sweep overwrites P_l (consumed by the forward sweep) in place;
//   * split-K partials of H in FP64, reduced in a fixed order by the
//     finalize kernel (deterministic, no atomics).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nnc.h"
#include "nnc_internal.h"

using namespace nnc;

namespace {

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

#define NNC_HIP(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      (ctx)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);             \
      return NNC_E_HIP;                                                                 \
    }                                                                                   \
  } while (0)

#define NNC_TRY(expr)        \
  do {                       \
    int rc_ = (expr);        \
    if (rc_ != NNC_OK) return rc_; \
  } while (0)

// Launch `call` bracketed by profiling events of kernel class `kind`.
#define NNC_LAUNCH(ctx, kind, call)  \
  do {                               \
    ProfRec pr_;                     \
    prof_begin((ctx), (kind), &pr_); \
    NNC_HIP((ctx), (call));          \
    prof_end((ctx), &pr_);           \
  } while (0)

int fail(Ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

void* dalloc(Net* net, size_t bytes) {
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  if (hipMemset(p, 0, bytes) != hipSuccess) {
    hipFree(p);
    return nullptr;
  }
  net->allocs.push_back(p);
  return p;
}

void free_net(Net* net) {
  if (!net) return;
  for (void* p : net->allocs) hipFree(p);
  if (net->part) hipFree(net->part);
  if (net->Hpart) hipFree(net->Hpart);
  delete net;
}

size_t dsize(DType t) { return t == DT_F64 ? 8 : (t == DT_F32 ? 4 : 2); }

int get_net(Ctx* c, int id, Net** out) {
  if (!c) return NNC_E_ARG;
  if (id < 0 || id >= (int)c->nets.size() || !c->nets[id])
    return fail(c, NNC_E_ARG, "invalid network handle");
  *out = c->nets[id];
  return NNC_OK;
}

// GEMM tiling choice before/without autotuning.
int pick_cfg(const Net* net, int M, int N, bool acc64) {
  const long long tiles128 = (long long)((M + 127) / 128) * ((N + 127) / 128);
  if (acc64) return tiles128 >= 256 ? 0 : 3;
  if (tiles128 >= 200) return 0;
  return 3;
}

// From this many points on, the primal pass and the FP64 adjoint run as MFMA
// GEMMs (the weight-streaming kernels carry at most 64 rows per pass over
// the weights, so many points would re-read every weight once per 64 rows).
constexpr int kGemmRows = 64;

// A GEMM in an explicit storage type (the FP64 adjoint of a lower-precision
// network): tuned tiling for that type and shape, else the heuristic; unsplit.
int gemm_dt(Ctx* c, Net* net, DType dt, GemmArgs g, int kind) {
  int cfg = -1;
  auto it = c->tuned.find(TuneKey{(int)dt, g.M, g.N, g.K, 0, 1});
  if (it != c->tuned.end()) cfg = it->second.cfg;
  if (c->forced_cfg[dt] >= 0) cfg = c->forced_cfg[dt];
  if (cfg < 0 || !gemm_cfg_supports(dt, cfg, false)) cfg = pick_cfg(net, g.M, g.N, false);
  if (g.kper <= 0) g.kper = g.K;
  NNC_LAUNCH(c, kind, launch_gemm(dt, cfg, false, g, 1, c->stream));
  return NNC_OK;
}

// Whether a GEMM may run as K slices (partials + fixed-order reduction):
// sweep and Jacobian epilogues (partials in FP32, in FP64 for FP64 GEMMs).
bool ksplit_ok(const Net* net, const GemmArgs& g, bool acc64, int splits) {
  (void)net;
  if (acc64 || splits != 1 || g.nbat > 0) return false;
  return g.epi == EPI_FWD_T || g.epi == EPI_FWD_G || g.epi == EPI_REV_G || g.epi == EPI_FWD_LS ||
         g.epi == EPI_FWD_LT || g.epi == EPI_JAC_R || g.epi == EPI_F64;
}

// Bytes per K-split partial element.
size_t part_size(const Net* net) { return net->ct == DT_F64 ? 8 : 4; }

// Launch one GEMM with tiling cfg, as ks K slices when ks > 1 and the
// workspace holds them (else unsplit).  Slices are whole K tiles.
hipError_t launch_gemm_ks(Net* net, GemmArgs g, bool acc64, int splits, int cfg, int ks, hipStream_t s) {
  if (g.kper <= 0) g.kper = g.K;
  if (ks > 1 && ksplit_ok(net, g, acc64, splits)) {
    const int BK = 128 / (int)net->csz;
    const int kper = ((g.K + ks - 1) / ks + BK - 1) / BK * BK;
    const int nsp = (g.K + kper - 1) / kper;
    if (nsp > 1 && (size_t)nsp * g.M * g.N * part_size(net) <= net->part_bytes) {
      GemmArgs gp = g;
      gp.epi = net->ct == DT_F64 ? EPI_PART64 : EPI_PART;
      gp.out0 = net->part;
      gp.ldo = g.N;
      gp.split_stride = (long long)g.M * g.N;
      gp.kper = kper;
      hipError_t e = launch_gemm(net->ct, cfg, false, gp, nsp, s);
      if (e != hipSuccess) return e;
      return launch_splitk_reduce(net->ct, g, net->part, nsp, s);
    }
  }
  return launch_gemm(net->ct, cfg, acc64, g, splits, s);
}

// Grow the K-split workspace to `bytes` (plan time only: network creation,
// autotuning, forcing a split; never inside an evaluation).
int ensure_part(Ctx* c, Net* net, size_t bytes) {
  if (bytes <= net->part_bytes) return NNC_OK;
  // a captured batch graph holds the old workspace address: drop it (the
  // next batched call re-plans and re-captures)
  free_batch(c);
  if (net->part) {
    NNC_HIP(c, hipDeviceSynchronize());
    hipFree(net->part);
    net->part = nullptr;
    net->part_bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return fail(c, NNC_E_NOMEM, "K-split workspace");
  net->part = p;
  net->part_bytes = bytes;
  return NNC_OK;
}

int plan_tangents(Net* net, int B, std::vector<PlannedGemm>& out);

// Workspace for the K splits the tuned table (or a forced split) asks for at
// B = 1 and B = max_points.
int size_part(Ctx* c, Net* net) {
  size_t need = 0;
  for (int B : {1, net->maxB}) {
    std::vector<PlannedGemm> plan;
    NNC_TRY(plan_tangents(net, B, plan));
    for (const PlannedGemm& p : plan) {
      if (!ksplit_ok(net, p.g, p.acc64, p.splits)) continue;
      int ks = 1;
      auto it = c->tuned.find(TuneKey{(int)net->ct, p.g.M, p.g.N, p.g.K, (int)p.acc64, p.splits});
      if (it != c->tuned.end()) ks = it->second.ksplit;
      if (c->forced_ksplit[net->ct] >= 1) ks = c->forced_ksplit[net->ct];
      if (ks > 1) need = std::max(need, (size_t)ks * p.g.M * p.g.N * part_size(net));
    }
  }
  return ensure_part(c, net, need);
}

// ---------------------------------------------------------------- Hessian methods
// Column offsets of each layer's tangents in the layer-sum buffers.
void layersum_layout(Net* net) {
  net->koff.assign(net->L + 2, 0);
  int k = 0;
  for (int l = 1; l <= net->Lt; ++l) {
    net->koff[l] = k;
    k += net->ly[l - 1].doutp;
  }
  net->Ktot = k;
}

// K splits of the symmetric layer-sum product at B points: enough work items
// for about four workgroups per CU, at most 8 slices, whole K tiles.
int ls_hsplits(const Net* net, int B) {
  const long long tt = (net->n + kSymTile - 1) / kSymTile;
  const long long tiles = (long long)B * tt * (tt + 1) / 2;
  long long sp = (1024 + tiles - 1) / tiles;
  sp = std::max(1LL, std::min(8LL, sp));
  const int ktiles = std::max(1, net->Ktot / (128 / (int)net->csz));
  return (int)std::min<long long>(sp, ktiles);
}

// The cheaper method by algorithmic flops of the work they do not share
// (both run the forward tangent sweep): the reverse sweep and H = W_1^T G_1,
// against the lower block triangle of the layer-sum product.
int auto_hess_method(const Net* net) {
  if (net->softmax_out) return NNC_HESS_LAYERSUM;  // the only method with the SoftMax coupling
  if (net->Lt == 0) return NNC_HESS_FOR;
  const double n = net->n;
  double rev = 2.0 * n * n * net->ly[0].doutp;
  for (int l = 2; l <= net->Lt; ++l) rev += 2.0 * n * net->ly[l - 1].doutp * net->ly[l - 2].doutp;
  const double tt = (net->n + kSymTile - 1) / kSymTile;
  const double ls = 2.0 * (tt * (tt + 1) / 2) * kSymTile * kSymTile * net->Ktot;
  return ls < rev ? NNC_HESS_LAYERSUM : NNC_HESS_FOR;
}

// Bytes of H partials the allocated methods need at any B <= max_points.
size_t hpart_need(const Net* net) {
  const size_t nn8 = (size_t)net->n * net->n * 8;
  size_t need = 0;
  if (net->for_bufs) need = (size_t)net->hsplit * net->maxB * nn8;
  if (net->ls_bufs)
    for (int B = 1; B <= net->maxB; ++B) need = std::max(need, (size_t)ls_hsplits(net, B) * B * nn8);
  return need;
}

// Workspace of Hessian method `method` (network creation, or a method change:
// plan time only).
int ensure_hess_bufs(Ctx* c, Net* net, int method) {
  const size_t N = (size_t)net->maxB * net->n;
  const int Lt = net->Lt;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* p = dalloc(net, bytes);
    if (!p) ok = false;
    return p;
  };
  if (Lt >= 2 && !net->P[1])
    for (int l = 1; l <= Lt - 1; ++l) net->P[l] = A(N * net->ly[l - 1].doutp * net->csz);
  if (method == NNC_HESS_FOR && !net->for_bufs) {
    for (int l = 2; l <= Lt - 1; ++l) net->T[l] = A(N * net->ly[l - 1].doutp * net->csz);
    if (Lt >= 1) net->Glast = A(N * net->ly[Lt - 1].doutp * net->csz);
    net->for_bufs = true;
  }
  if (method == NNC_HESS_LAYERSUM && !net->ls_bufs) {
    if (Lt >= 1) {
      net->TC = A(N * net->Ktot * net->csz);
      net->SC = A(N * net->Ktot * net->csz);
    }
    net->ls_bufs = true;
  }
  if (!ok) return fail(c, NNC_E_NOMEM, "Hessian workspace");
  const size_t need = std::max<size_t>(hpart_need(net), 16);
  if (need > net->hpart_bytes) {
    free_batch(c);  // a captured batch graph holds the old address
    if (net->Hpart) {
      NNC_HIP(c, hipDeviceSynchronize());
      hipFree(net->Hpart);
      net->Hpart = nullptr;
      net->hpart_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) return fail(c, NNC_E_NOMEM, "Hessian partials");
    net->Hpart = (double*)p;
    net->hpart_bytes = need;
  }
  return NNC_OK;
}

int gemm(Ctx* c, Net* net, int slot, GemmArgs g, bool acc64, int splits, int kind = NNC_KC_GEMM) {
  int cfg = -1, ks = 1;
  (void)slot;
  if (g.sym > 0) {  // symmetric layer-sum product: its tiling is fixed (square tiles of edge sym)
    NNC_LAUNCH(c, kind, launch_gemm(net->ct, kSymCfg, acc64, g, splits, c->stream));
    return NNC_OK;
  }
  auto it = c->tuned.find(TuneKey{(int)net->ct, g.M, g.N, g.K, (int)acc64, splits});
  if (it != c->tuned.end()) {
    cfg = it->second.cfg;
    ks = it->second.ksplit;
  }
  if (!acc64 && c->forced_cfg[net->ct] >= 0) cfg = c->forced_cfg[net->ct];
  if (!acc64 && c->forced_ksplit[net->ct] >= 1) ks = c->forced_ksplit[net->ct];
  if (cfg < 0 || !gemm_cfg_supports(net->ct, cfg, acc64)) cfg = pick_cfg(net, g.M, g.N, acc64);
  NNC_LAUNCH(c, kind, launch_gemm_ks(net, g, acc64, splits, cfg, ks, c->stream));
  return NNC_OK;
}

GemmArgs gemm_args(const void* A, long long lda, const void* B, long long ldb, int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.lda = lda;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.kper = K;
  g.rdiv = 1;
  return g;
}

SkinnyArgs skinny_args(const void* W, long long ldw, int N, int K, const void* X, long long ldx,
                       int rows, int epi) {
  SkinnyArgs a;
  memset(&a, 0, sizeof(a));
  a.W = W;
  a.ldw = ldw;
  a.N = N;
  a.K = K;
  a.X = X;
  a.ldx = ldx;
  a.rows = rows;
  a.epi = epi;
  a.rdiv = 1;
  return a;
}

int check_finite(Ctx* c, Net* net, const double* p, size_t count) {
  if (!c->debug_checks || !p || count == 0) return NNC_OK;
  NNC_HIP(c, launch_fill_zero(net->dflag, sizeof(int), c->stream));
  NNC_HIP(c, launch_check_finite(p, count, net->dflag, c->stream));
  int h = 0;
  NNC_HIP(c, hipMemcpyAsync(&h, net->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NNC_HIP(c, hipStreamSynchronize(c->stream));
  if (h) return fail(c, NNC_E_NONFINITE, "non-finite input");
  return NNC_OK;
}

// ---------------------------------------------------------------- the path
// FP64 adjoint step through layer l (W_l^T): zbar_l -> zbar_{l-1}, s_{l-1}.
SkinnyArgs adjoint_args(Net* net, int l, int B) {
  Layer& ly = net->ly[l - 1];
  Layer& lp = net->ly[l - 2];
  SkinnyArgs a = skinny_args(ly.WT, ly.doutp, lp.doutp, ly.doutp, ly.zbar, ly.doutp, B, SK_ADJ);
  a.Wp = ly.WTP;  // NULL for the output layer
  a.part = net->spart64;
  a.part_elems = net->spart64_elems;
  a.dtrue = lp.dout;
  a.act = lp.act;
  a.vec = lp.z;
  a.ldv = lp.doutp;
  a.out0 = lp.zbar;
  a.out1 = lp.s;
  a.ldo = lp.doutp;
  a.ldo1 = lp.doutp;
  return a;
}

// One point with float weights: the hidden-layer adjoint steps use the MFMA
// weight stream that can also carry the Jacobian rows (5..64 of them, the
// range in which the Jacobian uses that stream on its own).
bool reverse_stream_ok(const Net* net, int B) { return B == 1 && net->ct != DT_F64; }
bool reverse_fusable(const Net* net, int B) {
  return reverse_stream_ok(net, B) && net->L >= 3 && net->m > 4 && net->m <= 64;
}


// Per-point vectors the forward pass writes: the staged input [B][np] and,
// per layer l, z_l (FP64), a_l and sigma'_l ([B][d_l'] each; sigma'_L in
// FP64).  The network's own buffers, or a caller-provided carve-up.
struct FwdBufs {
  void* xin = nullptr;
  std::vector<double*> z;
  std::vector<void*> a, d1;
};

FwdBufs net_fwd_bufs(Net* net) {
  FwdBufs f;
  f.xin = net->xin;
  for (Layer& ly : net->ly) {
    f.z.push_back(ly.z);
    f.a.push_back(ly.a);
    f.d1.push_back(ly.d1);
  }
  return f;
}

// a1 + a2 + a3: stage x, primal forward, FP64 output layer (and residual).
// layer_events: record c->ev_layer[l - 1] on the stream once layer l's
// outputs (z_l, a_l, sigma'_l) are written, for work on the side stream.
int run_forward_bufs(Ctx* c, Net* net, int B, const double* x, const double* y, double* g, const FwdBufs& fb,
                     bool layer_events = false) {
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_cast_input(net->at, x, B, net->n, fb.xin, net->np, c->stream));
  const void* X = fb.xin;
  // many points: each hidden layer is one MFMA GEMM with the primal epilogue
  // (activations and weights in the same type; FP32 and FP64 networks)
  const bool gemm_fwd = B >= kGemmRows && net->ct == net->at;
  for (int l = 1; l < net->L; ++l) {
    Layer& ly = net->ly[l - 1];
    if (gemm_fwd) {
      GemmArgs gg = gemm_args(X, ly.dinp, ly.W, ly.dinp, B, ly.doutp, ly.dinp);
      gg.epi = EPI_PRIMAL;
      gg.out0 = fb.z[l - 1];
      gg.out1 = fb.a[l - 1];
      gg.out2 = fb.d1[l - 1];
      gg.ldo = ly.doutp;
      gg.bias64 = ly.b;
      gg.act = ly.act;
      gg.dtrue = ly.dout;
      NNC_TRY(gemm_dt(c, net, net->ct, gg, NNC_KC_SKINNY));
      X = fb.a[l - 1];
      continue;
    }
    SkinnyArgs a = skinny_args(ly.W, ly.dinp, ly.doutp, ly.dinp, X, ly.dinp, B, SK_PRIMAL);
    a.dtrue = ly.dout;
    a.act = ly.act;
    a.bias = ly.b;
    a.out0 = fb.z[l - 1];
    a.out1 = fb.a[l - 1];
    a.out2 = fb.d1[l - 1];
    a.ldo = ly.doutp;
    NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(net->ct, net->at, net->at, a, c->stream));
    X = fb.a[l - 1];
    if (layer_events) NNC_HIP(c, hipEventRecord(c->ev_layer[l - 1], c->stream));
  }
  Layer& lo = net->ly[net->L - 1];
  SkinnyArgs a = skinny_args(net->WL64, lo.dinp, net->m, lo.dinp, X, lo.dinp, B, SK_OUT);
  a.act = lo.act;
  a.bias = lo.b;
  a.out0 = fb.z[net->L - 1];
  a.out2 = fb.d1[net->L - 1];
  a.ldo = lo.doutp;
  a.out1 = g;
  a.ldo1 = net->m;
  a.y = y;
  NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(DT_F64, net->at, DT_F64, a, c->stream));
  if (net->softmax_out)  // p = softmax(z_L) in FP64 (in the output layer's sigma' slot), g = y - p
    NNC_LAUNCH(c, NNC_KC_OTHER, launch_softmax_out(fb.z[net->L - 1], B, net->m, lo.doutp, y, g,
                                                   (double*)fb.d1[net->L - 1], c->stream));
  if (layer_events) NNC_HIP(c, hipEventRecord(c->ev_layer[net->L - 1], c->stream));
  return NNC_OK;
}

int run_forward(Ctx* c, Net* net, int B, const double* x, const double* y, double* g) {
  return run_forward_bufs(c, net, B, x, y, g, net_fwd_bufs(net));
}

// Bytes of the forward pass's per-point vectors at B points, each carved at
// a 256-byte boundary (static-workspace variant of eval_g); fills fb when
// base is given.
size_t carve_fwd_bufs(const Net* net, int B, char* base, FwdBufs* fb) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  void* xin = take((size_t)B * net->np * net->asz);
  if (fb) fb->xin = xin;
  for (int l = 1; l <= net->L; ++l) {
    const Layer& ly = net->ly[l - 1];
    double* z = (double*)take((size_t)B * ly.doutp * 8);
    void* a = take((size_t)B * ly.doutp * net->asz);
    void* d1 = take((size_t)B * ly.doutp * (l == net->L ? 8 : net->asz));
    if (fb) {
      fb->z.push_back(z);
      fb->a.push_back(a);
      fb->d1.push_back(d1);
    }
  }
  return off;
}

// a4 + a5 at one point (reverse_fusable): each hidden layer's W^T is streamed
// once for the Jacobian rows and the FP64 adjoint row together.  Launch for
// launch the same arguments, kernels and rounding as run_jacobian followed
// by run_adjoint, so the results are the same bits.
int run_jacobian_adjoint(Ctx* c, Net* net, double* J, const double* lam) {
  const int L = net->L, m = net->m, n = net->n;
  Layer& lo = net->ly[L - 1];
  Layer& lp = net->ly[L - 2];
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_jac_seed(net->at, net->WL64, m, lp.dout, lo.dinp, lo.d1, lo.doutp, lp.d1,
                             lp.doutp, 1, net->R0, false, net->softmax_out, c->stream));
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_adj_seed(lam, lo.z, lo.act, 1, m, lo.doutp, lo.zbar, lo.s, (const double*)lo.d1,
                                              c->stream));
  {
    SkinnyArgs a = adjoint_args(net, L, 1);
    a.W = net->WLT64;  // the output layer's adjoint step stays in FP64 weights
    a.Wp = nullptr;
    NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(DT_F64, DT_F64, DT_F64, a, c->stream));
  }
  void* cur = net->R0;
  void* nxt = net->R1;
  for (int l = L - 1; l >= 2; --l) {
    Layer& ly = net->ly[l - 1];
    Layer& lprev = net->ly[l - 2];
    SkinnyArgs a = skinny_args(ly.WT, ly.doutp, lprev.doutp, ly.doutp, cur, ly.doutp, m, SK_JAC_R);
    a.Wp = ly.WTP;
    a.part = net->spart;
    a.part_elems = net->spart_elems;
    a.rdiv = m;
    a.vec = lprev.d1;
    a.ldv = lprev.doutp;
    a.out0 = nxt;
    a.ldo = lprev.doutp;
    const SkinnyArgs d = adjoint_args(net, l, 1);
    NNC_LAUNCH(c, NNC_KC_SKINNY, launch_reverse_stream(net->ct, a, d, c->stream));
    std::swap(cur, nxt);
  }
  Layer& l1 = net->ly[0];
  SkinnyArgs a = skinny_args(l1.WT, l1.doutp, n, l1.doutp, cur, l1.doutp, m, SK_JAC_OUT);
  a.Wp = l1.WTP;
  a.part = net->spart;
  a.part_elems = net->spart_elems;
  a.out0 = J;
  a.ldo = n;
  NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(net->ct, net->at, net->at, a, c->stream));
  return NNC_OK;
}

// a4: Jacobian by m reverse passes per point.
int run_jacobian(Ctx* c, Net* net, int B, double* J) {
  const int L = net->L, m = net->m, n = net->n;
  Layer& lo = net->ly[L - 1];
  if (L == 1) {
    NNC_LAUNCH(c, NNC_KC_OTHER, launch_jac_seed(net->at, net->WL64, m, n, lo.dinp, lo.d1, lo.doutp, nullptr, 0, B, J,
                               true, net->softmax_out, c->stream));
    return NNC_OK;
  }
  Layer& lp = net->ly[L - 2];
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_jac_seed(net->at, net->WL64, m, lp.dout, lo.dinp, lo.d1, lo.doutp, lp.d1,
                             lp.doutp, B, net->R0, false, net->softmax_out, c->stream));
  void* cur = net->R0;
  void* nxt = net->R1;
  const int rows = B * m;
  // Many rows (B*m >= 64): the reverse passes are a real GEMM, run on MFMA.
  const bool mfma = rows >= 64 && net->ct == net->at;
  for (int l = L - 1; l >= 2; --l) {
    Layer& ly = net->ly[l - 1];
    Layer& lprev = net->ly[l - 2];
    if (mfma) {
      GemmArgs g = gemm_args(cur, ly.doutp, ly.WT, ly.doutp, rows, lprev.doutp, ly.doutp);
      g.epi = EPI_JAC_R;
      g.rdiv = m;
      g.v0 = lprev.d1;
      g.ldv = lprev.doutp;
      g.out0 = nxt;
      g.ldo = lprev.doutp;
      NNC_TRY(gemm(c, net, -1, g, false, 1));
    } else {
      SkinnyArgs a = skinny_args(ly.WT, ly.doutp, lprev.doutp, ly.doutp, cur, ly.doutp, rows, SK_JAC_R);
      a.Wp = ly.WTP;
      a.part = net->spart;
      a.part_elems = net->spart_elems;
      a.rdiv = m;
      a.vec = lprev.d1;
      a.ldv = lprev.doutp;
      a.out0 = nxt;
      a.ldo = lprev.doutp;
      NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(net->ct, net->at, net->at, a, c->stream));
    }
    std::swap(cur, nxt);
  }
  Layer& l1 = net->ly[0];
  if (mfma) {
    GemmArgs g = gemm_args(cur, l1.doutp, l1.WT, l1.doutp, rows, n, l1.doutp);
    g.epi = EPI_F64;
    g.out0 = J;
    g.ldo = n;
    NNC_TRY(gemm(c, net, -1, g, false, 1));
    return NNC_OK;
  }
  SkinnyArgs a = skinny_args(l1.WT, l1.doutp, n, l1.doutp, cur, l1.doutp, rows, SK_JAC_OUT);
  a.Wp = l1.WTP;
  a.part = net->spart;
  a.part_elems = net->spart_elems;
  a.out0 = J;
  a.ldo = n;
  NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(net->ct, net->at, net->at, a, c->stream));
  return NNC_OK;
}

// a5: FP64 adjoint of lambda^T NN: zbar_l and s_l for every layer.
int run_adjoint(Ctx* c, Net* net, int B, const double* lam) {
  const int L = net->L;
  Layer& lo = net->ly[L - 1];
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_adj_seed(lam, lo.z, lo.act, B, net->m, lo.doutp, lo.zbar, lo.s,
                                              (const double*)lo.d1, c->stream));
  // many points: FP64 MFMA GEMMs against FP64 copies of W^T
  const bool gemm_adj = B >= kGemmRows;  // (copies exist whenever max_points >= kGemmRows)
  for (int l = L; l >= 2; --l) {
    Layer& ly = net->ly[l - 1];
    Layer& lp = net->ly[l - 2];
    const bool out_layer = (l == L);
    if (gemm_adj && (out_layer || ly.WT64)) {
      const double* W64 = out_layer ? net->WLT64 : ly.WT64;
      GemmArgs gg = gemm_args(ly.zbar, ly.doutp, W64, ly.doutp, B, lp.doutp, ly.doutp);
      gg.epi = EPI_ADJ64;
      gg.v0 = lp.z;
      gg.ldv = lp.doutp;
      gg.out0 = lp.zbar;
      gg.out1 = lp.s;
      gg.ldo = lp.doutp;
      gg.act = lp.act;
      gg.dtrue = lp.dout;
      NNC_TRY(gemm_dt(c, net, DT_F64, gg, NNC_KC_SKINNY));
      continue;
    }
    const void* W = out_layer ? (const void*)net->WLT64 : ly.WT;
    const DType wt = out_layer ? DT_F64 : net->ct;
    SkinnyArgs a = adjoint_args(net, l, B);
    if (!out_layer && reverse_stream_ok(net, B)) {
      // one point: the same stream (and rounding) as the fused Jacobian + adjoint pass
      SkinnyArgs none = skinny_args(ly.WT, ly.doutp, lp.doutp, ly.doutp, nullptr, ly.doutp, 0, SK_JAC_R);
      none.Wp = ly.WTP;
      NNC_LAUNCH(c, NNC_KC_SKINNY, launch_reverse_stream(wt, none, a, c->stream));
      continue;
    }
    a.W = W;
    if (out_layer) a.Wp = nullptr;
    NNC_LAUNCH(c, NNC_KC_SKINNY, launch_skinny(wt, DT_F64, DT_F64, a, c->stream));
  }
  return NNC_OK;
}

// a6 + a7: the GEMMs of the forward- and reverse-tangent sweeps and of H,
// as argument blocks (phase 0 forward, 1 reverse, 2 H; idx = step in phase).
// Layer sum: the forward sweep writes T_l and S_l = diag(s_l) T_l of every
// layer into one row per tangent column (layer l at column koff[l]) and P_l
// for the next product; H[b] = sum_k T[(b,i)][k] S[(b,j)][k] is one product
// per point over all layers at once (K = sum of the padded widths), only
// its lower block triangle, FP64 across K tiles, K split into slices that
// the finalize kernel adds in order.  defer_s: the sweep writes T_l and P_l
// only (it then needs no adjoint) and S is formed afterwards.
int plan_layersum(Net* net, int B, std::vector<PlannedGemm>& out, bool defer_s = false) {
  out.clear();
  const int n = net->n, Lt = net->Lt;
  const int N = B * n;
  if (Lt == 0) return NNC_OK;
  const bool fp64 = (net->ct == DT_F64);
  int slot = 0;
  for (int l = 1; l <= Lt - 1; ++l, ++slot) {
    Layer& nx = net->ly[l];  // layer l+1
    Layer& cu = net->ly[l - 1];
    GemmArgs g = gemm_args(net->P[l], cu.doutp, nx.W, nx.dinp, N, nx.doutp, cu.doutp);
    g.rdiv = n;
    g.epi = defer_s ? EPI_FWD_LT : EPI_FWD_LS;
    g.out0 = (char*)net->TC + (size_t)net->koff[l + 1] * net->csz;
    g.out2 = defer_s ? nullptr : (char*)net->SC + (size_t)net->koff[l + 1] * net->csz;
    g.ldo = net->Ktot;
    g.out1 = (l + 1 < Lt) ? net->P[l + 1] : nullptr;
    g.ldo1 = nx.doutp;
    g.v0 = nx.d1;
    g.v1 = nx.s;
    g.ldv = nx.doutp;
    out.push_back(PlannedGemm{0, l - 1, g, false, 1, slot});
  }
  GemmArgs g = gemm_args(net->TC, net->Ktot, net->SC, net->Ktot, n, n, net->Ktot);
  g.epi = EPI_H64;
  g.out0 = net->Hpart;
  g.ldo = n;
  g.split_stride = (long long)N * n;
  g.nbat = B;
  g.sym = kSymTile;
  g.bsA = (long long)n * net->Ktot;
  g.bsB = (long long)n * net->Ktot;
  g.bsO = (long long)n * n;
  const int BK = 128 / (int)net->csz;
  int splits = ls_hsplits(net, B);
  const int kper = round_up((net->Ktot + splits - 1) / splits, BK);
  splits = (net->Ktot + kper - 1) / kper;
  g.kper = kper;
  out.push_back(PlannedGemm{2, 0, g, !fp64, splits, slot});
  return NNC_OK;
}

int plan_tangents(Net* net, int B, std::vector<PlannedGemm>& out) {
  if (net->hess_method == NNC_HESS_LAYERSUM) return plan_layersum(net, B, out);
  out.clear();
  const int n = net->n, Lt = net->Lt;
  const int N = B * n;
  if (Lt == 0) return NNC_OK;
  Layer& l1 = net->ly[0];
  const bool fp64 = (net->ct == DT_F64);
  int slot = 0;
  // forward sweep: T_{l+1} = W_{l+1} (D_l T_l), stored as [N][d_{l+1}]
  for (int l = 1; l <= Lt - 1; ++l, ++slot) {
    Layer& nx = net->ly[l];  // layer l+1
    Layer& cu = net->ly[l - 1];
    GemmArgs g = gemm_args(net->P[l], cu.doutp, nx.W, nx.dinp, N, nx.doutp, cu.doutp);
    g.rdiv = n;
    g.ldo = nx.doutp;
    g.ldv = nx.doutp;
    if (l + 1 < Lt) {
      g.epi = EPI_FWD_T;
      g.out0 = net->T[l + 1];
      g.out1 = net->P[l + 1];
      g.v0 = nx.d1;
    } else {
      g.epi = EPI_FWD_G;
      g.out0 = net->Glast;
      g.v0 = nx.s;
    }
    out.push_back(PlannedGemm{0, l - 1, g, false, 1, slot});
  }
  // reverse sweep: G_{l-1} = D_{l-1} W_l^T G_l + diag(s_{l-1}) T_{l-1}
  for (int l = Lt; l >= 2; --l, ++slot) {
    Layer& cu = net->ly[l - 1];
    Layer& pv = net->ly[l - 2];
    const void* Gl = (l == Lt) ? net->Glast : net->P[l];
    GemmArgs g = gemm_args(Gl, cu.doutp, cu.WT, cu.doutp, N, pv.doutp, cu.doutp);
    g.rdiv = n;
    g.epi = EPI_REV_G;
    g.out0 = net->P[l - 1];
    g.ldo = pv.doutp;
    g.v0 = pv.d1;
    g.v1 = pv.s;
    g.ldv = pv.doutp;
    if (l - 1 == 1) {
      g.aux = l1.WT;
      g.auxmod = n;
    } else {
      g.aux = net->T[l - 1];
    }
    g.ldaux = pv.doutp;
    out.push_back(PlannedGemm{1, Lt - l, g, false, 1, slot});
  }
  // H rows (b, i): H[b][i][:] = G_1[(b,i)][:] W_1, accumulated in FP64.
  const void* G1 = (Lt == 1) ? net->Glast : net->P[1];
  GemmArgs g = gemm_args(G1, l1.doutp, l1.WT, l1.doutp, N, n, l1.doutp);
  g.epi = EPI_H64;
  g.out0 = net->Hpart;
  g.ldo = n;
  g.split_stride = (long long)N * n;
  const int BK = 128 / (int)net->csz;
  int splits = net->hsplit;
  const long long tiles = (long long)((N + 63) / 64) * ((n + 63) / 64);
  if (tiles >= 512) splits = 1;
  const int kper = round_up((l1.doutp + splits - 1) / splits, BK);
  splits = (l1.doutp + kper - 1) / kper;
  g.kper = kper;
  out.push_back(PlannedGemm{2, 0, g, !fp64, splits, slot});
  return NNC_OK;
}

// First tangent seed: P_1 = D_1 W_1 (or G_1 = diag(s_1) W_1 when Lt = 1).
int run_seed(Ctx* c, Net* net, int B, bool defer_s = false) {
  const int n = net->n;
  Layer& l1 = net->ly[0];
  if (net->Lt == 0) return NNC_OK;
  if (net->hess_method == NNC_HESS_LAYERSUM) {
    NNC_LAUNCH(c, NNC_KC_OTHER, launch_seed_layersum(net->ct, l1.WT, n, l1.doutp, l1.d1, l1.s, B, net->TC,
                                                      defer_s ? nullptr : net->SC, net->Ktot,
                                                      net->Lt >= 2 ? net->P[1] : nullptr, c->stream));
    return NNC_OK;
  }
  if (net->Lt == 1) {
    NNC_LAUNCH(c, NNC_KC_OTHER, launch_seed_tangent(net->ct, l1.WT, n, l1.doutp, l1.s, true, B, net->Glast, c->stream));
  } else {
    NNC_LAUNCH(c, NNC_KC_OTHER, launch_seed_tangent(net->ct, l1.WT, n, l1.doutp, l1.d1, net->ct == DT_F64, B, net->P[1], c->stream));
  }
  return NNC_OK;
}

// a8: sum split partials, symmetrise, add obj_factor * diag(q).
int run_finalize(Ctx* c, Net* net, int B, int splits, double obj, double* H, int symtile) {
  const int n = net->n;
  const double* q = net->q;
  if (net->Lt == 0) splits = 0;
  const bool sm = net->softmax_out && net->Lt > 0;
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_finalize_h(net->Hpart, splits, (long long)B * n * n, B, n, q ? obj : 0.0, q, H,
                                                symtile, sm ? net->usm : nullptr, sm ? net->vsm : nullptr,
                                                c->stream));
  return NNC_OK;
}

// SoftMax output: u = T_L^T p, v = T_L^T g from the output layer's tangents
// (the layer-sum forward sweep wrote them at column koff[L]).
int run_softmax_uv(Ctx* c, Net* net, int B) {
  if (!net->softmax_out || net->Lt == 0) return NNC_OK;
  Layer& lo = net->ly[net->L - 1];
  const void* TL = (const char*)net->TC + (size_t)net->koff[net->L] * net->csz;
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_softmax_uv(net->ct, TL, net->Ktot, B, net->n, net->m, lo.doutp,
                                                (const double*)lo.d1, lo.s, net->usm, net->vsm, c->stream));
  return NNC_OK;
}

// The planned GEMMs of phases lo..hi, in plan order; the H product's K
// splits and tile edge for the finalize kernel.
int run_planned(Ctx* c, Net* net, std::vector<PlannedGemm>& plan, int lo, int hi, int* splits, int* symtile) {
  for (PlannedGemm& p : plan) {
    if (p.phase < lo || p.phase > hi) continue;
    NNC_TRY(gemm(c, net, p.slot, p.g, p.acc64, p.splits, p.phase == 2 ? NNC_KC_GEMM_H : NNC_KC_GEMM));
    if (p.phase == 2) {
      *splits = p.splits;
      *symtile = p.g.sym;
    }
  }
  return NNC_OK;
}

int run_tangents(Ctx* c, Net* net, int B, double obj, double* H) {
  std::vector<PlannedGemm> plan;
  NNC_TRY(plan_tangents(net, B, plan));
  NNC_TRY(run_seed(c, net, B));
  int splits = 0, symtile = 0;
  NNC_TRY(run_planned(c, net, plan, 0, 2, &splits, &symtile));
  NNC_TRY(run_softmax_uv(c, net, B));
  return run_finalize(c, net, B, splits, obj, H, symtile);
}

// Whether the layer-sum forward sweep runs beside the reverse passes.  They
// must be weight streams (no GEMM, so no shared K-split workspace) and the
// layers must fit one scale launch.  And it must pay: the streams share the
// CUs with the sweep's GEMMs, which then run slower, so the streams' weight
// bytes at HBM rate must take at least a quarter of one point's sweep flops
// at the MFMA peak of its type (per point, so that every B below 64 takes
// the same path and a point gets the same bits alone or in a batch).  Measured with and without: 137M net FP32 448 vs
// 445 H/s (ratio 0.08: not taken), BF16 1576 -> 1683 (0.65); the deep,
// narrow net FP32 212 -> 242 (0.52), BF16 340 -> 445.
bool sweep_overlap_ok(const Ctx* c, const Net* net, int B, bool jac) {
  if (!c->side || net->hess_method != NNC_HESS_LAYERSUM || net->Lt == 0) return false;
  if (net->Lt > kMaxScaleLayers || B >= kGemmRows) return false;
  if (jac && !reverse_fusable(net, B) && (long long)B * net->m >= 64) return false;
  double wbytes = 0.0, flops = 0.0;
  for (int l = 2; l <= net->Lt; ++l) {
    const double w = (double)net->ly[l - 1].dout * net->ly[l - 1].din;
    wbytes += w * net->csz;
    flops += 2.0 * net->n * w;
  }
  const double peak = net->ct == DT_F64 ? 78.6e12 : net->ct == DT_F32 ? 157.3e12 : 2516.6e12;
  return wbytes / 5.0e12 >= 0.25 * flops / peak;
}

// S_l = diag(s_l) T_l of every layer, once the sweep (T) and the adjoint (s)
// are both done.
int run_scale(Ctx* c, Net* net, int B) {
  LsScaleArgs a;
  memset(&a, 0, sizeof(a));
  a.Tc = net->TC;
  a.Sc = net->SC;
  a.ld = net->Ktot;
  a.rows = B * net->n;
  a.n = net->n;
  a.layers = net->Lt;
  for (int l = 1; l <= net->Lt; ++l) {
    a.s[l - 1] = net->ly[l - 1].s;
    a.koff[l - 1] = net->koff[l];
    a.dp[l - 1] = net->ly[l - 1].doutp;
  }
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_scale_layersum(net->ct, a, c->stream));
  return NNC_OK;
}

// Layer-sum Hessian with its forward sweep on the side stream.  The sweep
// needs only the forward pass (S = diag(s) T is formed afterwards), so it
// runs beside `reverse` (the Jacobian and / or adjoint weight streams,
// memory-bound) on the main stream; then S, the H product and the finalize
// on the main stream.  The forward pass (x, y, g) is run here.  On a
// shallow network (L <= 8) the sweep also starts layer by layer: the seed
// once layer 1 of the forward pass is done and each sweep GEMM once the
// layer whose sigma' its epilogue applies is done, beside the rest of the
// forward pass (137M net BF16: 1693 -> 1761 H evals/s).  On the 39-layer
// net that interleaving measured slower (BF16 443 -> 405, FP32 243 -> 237),
// so there the sweep waits for the whole forward pass.
template <typename Rev>
int run_hess_overlapped(Ctx* c, Net* net, int B, const double* x, const double* y, double* g, double obj,
                        double* H, Rev reverse) {
  std::vector<PlannedGemm> plan;
  NNC_TRY(plan_layersum(net, B, plan, true));
  while ((int)c->ev_layer.size() < net->L) {
    hipEvent_t e = nullptr;
    NNC_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->ev_layer.push_back(e);
  }
  NNC_HIP(c, hipEventRecord(c->ev_fork, c->stream));
  NNC_HIP(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  const bool by_layer = net->L <= 8;
  NNC_TRY(run_forward_bufs(c, net, B, x, y, g, net_fwd_bufs(net), by_layer));
  if (!by_layer) NNC_HIP(c, hipEventRecord(c->ev_layer[net->L - 1], c->stream));  // the whole forward pass
  const hipStream_t main = c->stream;
  int splits = 0, symtile = 0;
  c->stream = c->side;
  hipError_t er = hipStreamWaitEvent(c->side, c->ev_layer[by_layer ? 0 : net->L - 1], 0);
  int rc = er == hipSuccess ? run_seed(c, net, B, true) : NNC_E_HIP;
  for (PlannedGemm& p : plan) {
    if (rc != NNC_OK || er != hipSuccess) break;
    if (p.phase != 0) continue;
    // sweep step idx writes T_{idx+2} with sigma' of layer idx + 2
    if (by_layer) er = hipStreamWaitEvent(c->side, c->ev_layer[p.idx + 1], 0);
    if (er == hipSuccess) rc = gemm(c, net, p.slot, p.g, p.acc64, p.splits, NNC_KC_GEMM);
  }
  const hipError_t ej = hipEventRecord(c->ev_join, c->side);
  c->stream = main;
  NNC_TRY(rc);
  NNC_HIP(c, er);
  NNC_HIP(c, ej);
  rc = reverse();
  NNC_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));  // joined before any return
  NNC_TRY(rc);
  NNC_TRY(run_scale(c, net, B));
  NNC_TRY(run_planned(c, net, plan, 2, 2, &splits, &symtile));
  NNC_TRY(run_softmax_uv(c, net, B));
  return run_finalize(c, net, B, splits, obj, H, symtile);
}

// ---------------------------------------------------------------- static workspace
// Workspace of nnc_eval_g_static: a fixed device array that every GPU the
// library runs on holds from code-object load to process exit, so that the
// entry point never allocates.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in symbol): its device address
// is looked up once per device, with that device current, when a context
// is created there, and kept per device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's workspace (the current device must be
// `device`); NNC_E_HIP if the lookup fails.
int resolve_scratch(Ctx* c, int device) {
  if (device < 0 || device >= kMaxDevices) return fail(c, NNC_E_UNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, NNC_E_HIP, std::string("hipGetSymbolAddress(static workspace) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  c->scratch = g_scratch_ptr[device];
  return NNC_OK;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

const char* nnc_strerror(int status) {
  switch (status) {
    case NNC_OK: return "ok";
    case NNC_E_ARG: return "invalid argument";
    case NNC_E_SHAPE: return "invalid shape";
    case NNC_E_NOMEM: return "out of device memory";
    case NNC_E_HIP: return "HIP runtime error";
    case NNC_E_NONFINITE: return "non-finite input";
    case NNC_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

int nnc_create(int device, void* hip_stream, nnc_ctx* out) {
  if (!out) return NNC_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return NNC_E_HIP;
  if (hipSetDevice(device) != hipSuccess) return NNC_E_HIP;
  Ctx* c = new Ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (resolve_scratch(c, device) != NNC_OK) {
    delete c;
    return NNC_E_HIP;
  }
  const char* dbg = getenv("NNC_DEBUG_CHECKS");
  c->debug_checks = dbg && dbg[0] && dbg[0] != '0';
  // the side stream of the layer-sum sweep (NNC_SWEEP_OVERLAP=0: none, the
  // whole evaluation on the caller's stream)
  const char* ov = getenv("NNC_SWEEP_OVERLAP");
  if (!(ov && ov[0] == '0')) {
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
      if (c->side) hipStreamDestroy(c->side);
      if (c->ev_fork) hipEventDestroy(c->ev_fork);
      if (c->ev_join) hipEventDestroy(c->ev_join);
      delete c;
      return NNC_E_HIP;
    }
  }
  load_tune_cache(c);
  *out = (nnc_ctx)c;
  return NNC_OK;
}

int nnc_destroy(nnc_ctx ctx) {
  if (!ctx) return NNC_OK;
  Ctx* c = (Ctx*)ctx;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
    hipEventDestroy(c->ev_fork);
    hipEventDestroy(c->ev_join);
  }
  for (hipEvent_t e : c->ev_layer) hipEventDestroy(e);
  for (Net* n : c->nets) free_net(n);
  for (hipEvent_t e : c->evpool) hipEventDestroy(e);
  free_trainers(c);
  free_kkts(c);
  free_batch(c);
  delete c;
  return NNC_OK;
}

int nnc_set_stream(nnc_ctx ctx, void* hip_stream) {
  if (!ctx) return NNC_E_ARG;
  ((Ctx*)ctx)->stream = (hipStream_t)hip_stream;
  return NNC_OK;
}

const char* nnc_last_error(nnc_ctx ctx) {
  if (!ctx) return "null context";
  return ((Ctx*)ctx)->err.c_str();
}

int nnc_net_create(nnc_ctx ctx, int L, const int* dims, const int* acts, const double* const* W,
                   const double* const* b, int prec, int max_points, int* net_out) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !dims || !acts || !W || !net_out) return fail(c, NNC_E_ARG, "null argument");
  if (L < 1 || max_points < 1) return fail(c, NNC_E_SHAPE, "L and max_points must be >= 1");
  for (int l = 0; l <= L; ++l)
    if (dims[l] < 1) return fail(c, NNC_E_SHAPE, "layer widths must be >= 1");
  for (int l = 0; l < L; ++l) {
    if (acts[l] < NNC_IDENTITY || acts[l] > NNC_SOFTMAX) return fail(c, NNC_E_ARG, "bad activation");
    if (acts[l] == NNC_SOFTMAX && l != L - 1) return fail(c, NNC_E_ARG, "SoftMax only on the output layer");
    if (!W[l]) return fail(c, NNC_E_ARG, "null weight matrix");
  }
  if (prec != NNC_FP64 && prec != NNC_FP32 && prec != NNC_BF16) return fail(c, NNC_E_ARG, "bad precision");
  NNC_HIP(c, hipSetDevice(c->device));

  Net* net = new Net();
  net->L = L;
  net->n = dims[0];
  net->m = dims[L];
  net->np = round_up(dims[0], 64);
  net->prec = prec;
  net->maxB = max_points;
  net->ct = prec == NNC_FP64 ? DT_F64 : (prec == NNC_FP32 ? DT_F32 : DT_BF16);
  net->at = prec == NNC_FP64 ? DT_F64 : DT_F32;
  net->csz = dsize(net->ct);
  net->asz = dsize(net->at);
  net->Lt = acts[L - 1] == NNC_IDENTITY ? L - 1 : L;
  net->softmax_out = acts[L - 1] == NNC_SOFTMAX;
  net->ly.resize(L);
  const int B = max_points;
  bool ok = true;
  auto A = [&](size_t bytes) {
    void* p = dalloc(net, bytes);
    if (!p) ok = false;
    return p;
  };
  size_t maxdp = 0;
  for (int l = 1; l <= L; ++l) {
    Layer& ly = net->ly[l - 1];
    ly.din = dims[l - 1];
    ly.dout = dims[l];
    ly.dinp = l == 1 ? net->np : round_up(dims[l - 1], 64);
    ly.doutp = round_up(dims[l], 64);
    ly.act = acts[l - 1];
    maxdp = std::max(maxdp, (size_t)ly.doutp);
    ly.W = A((size_t)ly.doutp * ly.dinp * net->csz);
    ly.WT = A((size_t)ly.dinp * ly.doutp * net->csz);
    // hidden layers: W^T also in the MFMA weight stream's read order (one
    // contiguous KiB per wave load; dinp is a multiple of 16)
    if (l < L) ly.WTP = A((size_t)ly.dinp * ly.doutp * net->csz);
    ly.b = (double*)A((size_t)ly.doutp * 8);
    ly.z = (double*)A((size_t)B * ly.doutp * 8);
    ly.a = A((size_t)B * ly.doutp * net->asz);
    ly.d1 = A((size_t)B * ly.doutp * (l == L ? 8 : net->asz));
    ly.zbar = (double*)A((size_t)B * ly.doutp * 8);
    ly.s = (double*)A((size_t)B * ly.doutp * 8);
    if (B >= kGemmRows && l < L) ly.WT64 = net->ct == DT_F64 ? (double*)ly.WT : (double*)A((size_t)ly.dinp * ly.doutp * 8);
  }
  // GEMM operands are addressed by 32-bit byte offsets (buffer loads whose
  // out-of-range offset is 2^31): every operand stays below 2 GiB.
  const unsigned long long wsz = B >= kGemmRows ? 8 : net->csz;  // FP64 adjoint operands
  if ((unsigned long long)B * net->n * maxdp * net->csz >= (1ull << 31) ||
      (unsigned long long)B * net->m * maxdp * net->csz >= (1ull << 31) ||
      (unsigned long long)B * maxdp * wsz >= (1ull << 31) ||
      (unsigned long long)maxdp * maxdp * wsz >= (1ull << 31)) {
    free_net(net);
    return fail(c, NNC_E_SHAPE, "max_points * n * width exceeds 2 GiB per GEMM operand");
  }
  Layer& lo = net->ly[L - 1];
  net->WL64 = (double*)A((size_t)lo.doutp * lo.dinp * 8);  // rows >= m are zero
  net->WLT64 = (double*)A((size_t)lo.dinp * lo.doutp * 8);
  net->xin = A((size_t)B * net->np * net->asz);
  net->P.assign(L + 1, nullptr);
  net->T.assign(L + 1, nullptr);
  net->hsplit = 4;
  layersum_layout(net);
  net->hess_method = auto_hess_method(net);
  net->R0 = A((size_t)B * net->m * maxdp * net->asz);
  net->R1 = A((size_t)B * net->m * maxdp * net->asz);
  net->dflag = (int*)A(16);
  if (net->at == DT_F32) {  // K slices of the MFMA weight streams: up to 16 slices of 64 rows x widest W^T
    size_t maxn = 0;
    for (int l = 1; l <= L; ++l) maxn = std::max(maxn, (size_t)net->ly[l - 1].dinp);
    net->spart_elems = 16LL * 64 * (long long)maxn;
    net->spart64_elems = 16LL * (long long)maxn;
    net->spart = (float*)A((size_t)net->spart_elems * 4);
    net->spart64 = (double*)A((size_t)net->spart64_elems * 8);
  }
  if (net->softmax_out) {
    net->usm = (double*)A((size_t)B * net->n * 8);
    net->vsm = (double*)A((size_t)B * net->n * 8);
  }
  net->tune.assign(2 * L + 2, -1);
  if (!ok) {
    free_net(net);
    return fail(c, NNC_E_NOMEM, "device allocation failed");
  }
  {
    const int rc = ensure_hess_bufs(c, net, net->hess_method);  // tangent workspace, H partials
    if (rc != NNC_OK) {
      free_net(net);
      return rc;
    }
  }

  // Upload and convert the weights (FP64 host -> padded compute-type copies).
  size_t maxw = 0;
  for (int l = 1; l <= L; ++l) maxw = std::max(maxw, (size_t)dims[l] * dims[l - 1]);
  double* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, maxw * 8);
  if (e != hipSuccess) {
    free_net(net);
    return fail(c, NNC_E_NOMEM, "device allocation failed (weight staging)");
  }
  int rc = NNC_OK;
  for (int l = 1; l <= L && rc == NNC_OK; ++l) {
    Layer& ly = net->ly[l - 1];
    const size_t cnt = (size_t)ly.dout * ly.din;
    if (hipMemcpy(tmp, W[l - 1], cnt * 8, hipMemcpyHostToDevice) != hipSuccess ||
        launch_convert_weights(net->ct, tmp, ly.dout, ly.din, ly.W, ly.doutp, ly.dinp, false, 0) != hipSuccess ||
        launch_convert_weights(net->ct, tmp, ly.dout, ly.din, ly.WT, ly.doutp, ly.dinp, true, 0) != hipSuccess ||
        (ly.WTP && launch_pack_fragments(net->ct, ly.WT, ly.doutp, ly.dinp, ly.doutp, ly.WTP, 0) != hipSuccess)) {
      rc = fail(c, NNC_E_HIP, "weight upload failed");
      break;
    }
    if (ly.WT64 && net->ct != DT_F64 &&
        launch_convert_weights(DT_F64, tmp, ly.dout, ly.din, ly.WT64, ly.doutp, ly.dinp, true, 0) != hipSuccess) {
      rc = fail(c, NNC_E_HIP, "weight upload failed");
      break;
    }
    if (l == L) {
      if (launch_convert_weights(DT_F64, tmp, ly.dout, ly.din, net->WL64, ly.doutp, ly.dinp, false, 0) != hipSuccess ||
          launch_convert_weights(DT_F64, tmp, ly.dout, ly.din, net->WLT64, ly.doutp, ly.dinp, true, 0) != hipSuccess) {
        rc = fail(c, NNC_E_HIP, "weight upload failed");
        break;
      }
    }
    if (b && b[l - 1]) {
      if (hipMemcpy(ly.b, b[l - 1], (size_t)ly.dout * 8, hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(c, NNC_E_HIP, "bias upload failed");
        break;
      }
    }
    if (hipDeviceSynchronize() != hipSuccess) rc = fail(c, NNC_E_HIP, "weight conversion failed");
  }
  hipFree(tmp);
  if (rc == NNC_OK) rc = size_part(c, net);  // K-split workspace the tuned table asks for
  if (rc != NNC_OK) {
    free_net(net);
    return rc;
  }
  c->nets.push_back(net);
  *net_out = (int)c->nets.size() - 1;
  return NNC_OK;
}

int nnc_net_destroy(nnc_ctx ctx, int id) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(get_net(c, id, &net));
  hipStreamSynchronize(c->stream);
  free_net(net);
  c->nets[id] = nullptr;
  return NNC_OK;
}

int nnc_net_set_objective_diag(nnc_ctx ctx, int id, const double* q) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(get_net(c, id, &net));
  // the finalize launches of a captured batch graph carry the diagonal's
  // address: re-plan on the next batched call
  if (net->q != q) free_batch(c);
  net->q = q;
  return NNC_OK;
}

int nnc_net_info(nnc_ctx ctx, int id, int* L, int* n, int* m, int* prec, int* max_points) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(get_net(c, id, &net));
  if (L) *L = net->L;
  if (n) *n = net->n;
  if (m) *m = net->m;
  if (prec) *prec = net->prec;
  if (max_points) *max_points = net->maxB;
  return NNC_OK;
}

int nnc_net_set_hess_method(nnc_ctx ctx, int id, int method) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(get_net(c, id, &net));
  if (method != NNC_HESS_AUTO && method != NNC_HESS_FOR && method != NNC_HESS_LAYERSUM)
    return fail(c, NNC_E_ARG, "unknown Hessian method");
  const int m = method == NNC_HESS_AUTO ? auto_hess_method(net) : method;
  if (net->softmax_out && m != NNC_HESS_LAYERSUM)
    return fail(c, NNC_E_UNSUPPORTED, "a SoftMax output needs the layer-sum Hessian method");
  NNC_HIP(c, hipSetDevice(c->device));
  NNC_TRY(ensure_hess_bufs(c, net, m));
  if (m != net->hess_method) {
    free_batch(c);  // batched launches are planned per method
    net->hess_method = m;
    NNC_TRY(size_part(c, net));
  }
  return NNC_OK;
}

int nnc_net_hess_method(nnc_ctx ctx, int id, int* method) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(get_net(c, id, &net));
  if (!method) return fail(c, NNC_E_ARG, "null method");
  *method = net->hess_method;
  return NNC_OK;
}

static int eval_prologue(Ctx* c, int id, int B, Net** net) {
  NNC_TRY(get_net(c, id, net));
  if (B < 0 || B > (*net)->maxB) return fail(c, NNC_E_SHAPE, "B outside [0, max_points]");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NNC_E_HIP, "hipSetDevice failed");
  return NNC_OK;
}

int nnc_eval_g(nnc_ctx ctx, int id, int B, const double* x, const double* y, double* g) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(eval_prologue(c, id, B, &net));
  if (B == 0) return NNC_OK;
  if (!x || !g) return fail(c, NNC_E_ARG, "null x or g");
  NNC_TRY(check_finite(c, net, x, (size_t)B * net->n));
  return run_forward(c, net, B, x, y, g);
}

int nnc_eval_g_static(nnc_ctx ctx, int id, int B, const double* x, const double* y, double* g) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(eval_prologue(c, id, B, &net));
  if (B == 0) return NNC_OK;
  if (!x || !g) return fail(c, NNC_E_ARG, "null x or g");
  if (!c->scratch) return fail(c, NNC_E_HIP, "static workspace not resolved for this device");
  const size_t need = carve_fwd_bufs(net, B, nullptr, nullptr);
  if (need > kStaticScratchBytes)
    return fail(c, NNC_E_SHAPE, "B points of this network need " + std::to_string(need) +
                                    " bytes of forward-pass vectors, above the 64 MiB static workspace");
  FwdBufs fb;
  carve_fwd_bufs(net, B, (char*)c->scratch, &fb);
  return run_forward_bufs(c, net, B, x, y, g, fb);
}

int nnc_eval_jac_g(nnc_ctx ctx, int id, int B, const double* x, double* J) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(eval_prologue(c, id, B, &net));
  if (B == 0) return NNC_OK;
  if (!x || !J) return fail(c, NNC_E_ARG, "null x or J");
  NNC_TRY(check_finite(c, net, x, (size_t)B * net->n));
  NNC_TRY(run_forward(c, net, B, x, nullptr, nullptr));
  return run_jacobian(c, net, B, J);
}

int nnc_eval_hess_lag(nnc_ctx ctx, int id, int B, const double* x, double obj_factor,
                      const double* lambda, double* H) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(eval_prologue(c, id, B, &net));
  if (B == 0) return NNC_OK;
  if (!x || !lambda || !H) return fail(c, NNC_E_ARG, "null x, lambda or H");
  NNC_TRY(check_finite(c, net, x, (size_t)B * net->n));
  NNC_TRY(check_finite(c, net, lambda, (size_t)B * net->m));
  if (sweep_overlap_ok(c, net, B, false))
    return run_hess_overlapped(c, net, B, x, nullptr, nullptr, obj_factor, H,
                               [&] { return run_adjoint(c, net, B, lambda); });
  NNC_TRY(run_forward(c, net, B, x, nullptr, nullptr));
  NNC_TRY(run_adjoint(c, net, B, lambda));
  return run_tangents(c, net, B, obj_factor, H);
}

int nnc_eval(nnc_ctx ctx, int id, int B, const double* x, const double* y, double obj_factor,
             const double* lambda, double* g, double* J, double* H) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  NNC_TRY(eval_prologue(c, id, B, &net));
  if (!g && !J && !H) return fail(c, NNC_E_ARG, "no output requested");
  if (B == 0) return NNC_OK;
  if (!x) return fail(c, NNC_E_ARG, "null x");
  if (H && !lambda) return fail(c, NNC_E_ARG, "H requested without lambda");
  NNC_TRY(check_finite(c, net, x, (size_t)B * net->n));
  if (H) NNC_TRY(check_finite(c, net, lambda, (size_t)B * net->m));
  if (H && sweep_overlap_ok(c, net, B, J != nullptr)) {
    return run_hess_overlapped(c, net, B, x, g ? y : nullptr, g, obj_factor, H, [&]() -> int {
      if (J && reverse_fusable(net, B)) return run_jacobian_adjoint(c, net, J, lambda);
      if (J) NNC_TRY(run_jacobian(c, net, B, J));
      return run_adjoint(c, net, B, lambda);
    });
  }
  NNC_TRY(run_forward(c, net, B, x, g ? y : nullptr, g));
  if (J && H && reverse_fusable(net, B)) {
    NNC_TRY(run_jacobian_adjoint(c, net, J, lambda));
    return run_tangents(c, net, B, obj_factor, H);
  }
  if (J) NNC_TRY(run_jacobian(c, net, B, J));
  if (H) {
    NNC_TRY(run_adjoint(c, net, B, lambda));
    NNC_TRY(run_tangents(c, net, B, obj_factor, H));
  }
  return NNC_OK;
}

int nnc_hess_pack_lower(nnc_ctx ctx, int B, int n, const double* H, double* Hp) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (B < 0 || n < 1) return fail(c, NNC_E_SHAPE, "B < 0 or n < 1");
  if (B == 0) return NNC_OK;
  if (!H || !Hp) return fail(c, NNC_E_ARG, "null H or Hp");
  if (H == Hp) return fail(c, NNC_E_ARG, "Hp must not alias H");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NNC_E_HIP, "hipSetDevice failed");
  NNC_LAUNCH(c, NNC_KC_OTHER, launch_pack_lower(H, B, n, Hp, c->stream));
  return NNC_OK;
}

int nnc_gemm_config_count(void) { return gemm_num_cfgs(); }

int nnc_set_gemm_config(nnc_ctx ctx, int prec, int config) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (prec != NNC_FP64 && prec != NNC_FP32 && prec != NNC_BF16) return fail(c, NNC_E_ARG, "bad precision");
  const DType dt = prec == NNC_FP64 ? DT_F64 : (prec == NNC_FP32 ? DT_F32 : DT_BF16);
  if (config < -1 || config >= gemm_num_cfgs()) return fail(c, NNC_E_ARG, "unknown GEMM config");
  c->forced_cfg[dt] = config;
  free_batch(c);  // batched launches are planned with the tiling: re-plan on the next call
  return NNC_OK;
}

int nnc_set_gemm_ksplit(nnc_ctx ctx, int prec, int ksplit) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (prec < NNC_FP64 || prec > NNC_BF16) return fail(c, NNC_E_ARG, "unknown precision");
  if (ksplit != -1 && (ksplit < 1 || ksplit > 8)) return fail(c, NNC_E_ARG, "ksplit outside -1, 1..8");
  const DType t = prec == NNC_FP64 ? DT_F64 : prec == NNC_FP32 ? DT_F32 : DT_BF16;
  c->forced_ksplit[t] = ksplit;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NNC_E_HIP, "hipSetDevice failed");
  free_batch(c);
  for (Net* net : c->nets)
    if (net && net->ct == t) NNC_TRY(size_part(c, net));
  return NNC_OK;
}

int nnc_profile(nnc_ctx ctx, int enable) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (enable) {
    NNC_HIP(c, hipSetDevice(c->device));
    while (c->evpool.size() < 8192) {
      hipEvent_t e;
      NNC_HIP(c, hipEventCreate(&e));
      c->evpool.push_back(e);
    }
    NNC_HIP(c, hipStreamSynchronize(c->stream));
    c->recs.clear();
    c->evused = 0;
  }
  c->prof = enable != 0;
  return NNC_OK;
}

int nnc_profile_classes(nnc_ctx ctx, int class_mask) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (class_mask < 0 || class_mask > 0xF) return fail(c, NNC_E_ARG, "class mask outside 0..0xF");
  c->prof_mask = class_mask;
  return NNC_OK;
}

int nnc_profile_read(nnc_ctx ctx, int kind, double* total_ms, long long* launches) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (kind < NNC_KC_GEMM || kind > NNC_KC_GEMM_H) return fail(c, NNC_E_ARG, "bad kernel class");
  NNC_HIP(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  long long cnt = 0;
  for (const ProfRec& r : c->recs) {
    if (r.kind != kind) continue;
    float ms = 0.f;
    NNC_HIP(c, hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    ++cnt;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = cnt;
  return NNC_OK;
}

}  // extern "C"

namespace nnc {
int prof_begin(Ctx* c, int kind, ProfRec* r) {
  r->kind = -1;
  if (!c->prof || !((c->prof_mask >> kind) & 1) || c->evused + 2 > c->evpool.size()) return 0;
  r->a = c->evpool[c->evused++];
  r->b = c->evpool[c->evused++];
  r->kind = kind;
  hipEventRecord(r->a, c->stream);
  return 1;
}
void prof_end(Ctx* c, ProfRec* r) {
  if (r->kind < 0) return;
  hipEventRecord(r->b, c->stream);
  c->recs.push_back(*r);
}
}  // namespace nnc

// ---------------------------------------------------------------- internal API for the
// batching, autotuning and training modules
namespace nnc {
int internal_get_net(Ctx* c, int id, Net** out) { return get_net(c, id, out); }
int internal_forward(Ctx* c, Net* net, int B, const double* x, const double* y, double* g) {
  return run_forward(c, net, B, x, y, g);
}
int internal_jacobian(Ctx* c, Net* net, int B, double* J) { return run_jacobian(c, net, B, J); }
int internal_adjoint(Ctx* c, Net* net, int B, const double* lam) { return run_adjoint(c, net, B, lam); }
int internal_tangents(Ctx* c, Net* net, int B, double obj, double* H) {
  return run_tangents(c, net, B, obj, H);
}
int internal_plan_tangents(Net* net, int B, std::vector<PlannedGemm>& out) {
  return plan_tangents(net, B, out);
}
int internal_seed(Ctx* c, Net* net, int B) { return run_seed(c, net, B); }
hipError_t internal_launch_gemm_ks(Net* net, GemmArgs g, bool acc64, int splits, int cfg, int ks,
                                   hipStream_t s) {
  return launch_gemm_ks(net, g, acc64, splits, cfg, ks, s);
}
bool internal_ksplit_ok(const Net* net, const GemmArgs& g, bool acc64, int splits) {
  return ksplit_ok(net, g, acc64, splits);
}
int internal_ensure_part(Ctx* c, Net* net, size_t bytes) { return ensure_part(c, net, bytes); }
int internal_finalize(Ctx* c, Net* net, int B, int splits, double obj, double* H, int symtile) {
  return run_finalize(c, net, B, splits, obj, H, symtile);
}
int internal_softmax_uv(Ctx* c, Net* net, int B) { return run_softmax_uv(c, net, B); }
int internal_pick_cfg(const Net* net, int M, int N, bool acc64) { return pick_cfg(net, M, N, acc64); }
}  // namespace nnc
