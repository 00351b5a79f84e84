// Batched multi-network evaluation: many points and several networks in one
// pass, as persistent grouped launches captured into a HIP graph.
//
// For a job list (network, B points, x, lambda, outputs) the call
//   * runs each network's primal forward, FP64 output layer, Jacobian and
//     FP64 adjoint (weight-streaming / small kernels, one per network);
//   * runs the tangent sweeps as ONE persistent grouped GEMM launch per
//     sweep step: forward step s of every network that has one, then
//     reverse step r of every network, then every H product -- the tiles of
//     all networks share one grid sized to the chip, ordered by cost, so the
//     short networks fill the gaps of the long one;
//   * symmetrises each H.
// The whole sequence is captured once into a HIP graph (on a private
// capture stream) and replayed on the context's stream while the job list
// (networks, point counts, pointers, objective factors) stays the same;
// any change re-plans and re-captures.  Planning uploads the grouped
// argument tables (device memory allocated then, never during a replay).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/nnc.h"
#include "nnc_internal.h"

namespace nnc {

namespace {

struct GroupLaunch {
  int cfg = 0;
  bool acc64 = false;
  int ngroups = 0;
  int grid = 0;
  GemmArgs* dargs = nullptr;
  int* doffs = nullptr;
};

struct BatchPlan {
  std::vector<nnc_job> jobs;
  std::vector<GroupLaunch> launches;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> allocs;
};

struct BatchState {
  hipStream_t cap = nullptr;
  BatchPlan* plan = nullptr;
};

void free_plan(BatchPlan* p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  for (void* a : p->allocs) hipFree(a);
  delete p;
}

bool same_jobs(const std::vector<nnc_job>& a, int n, const nnc_job* b) {
  if ((int)a.size() != n) return false;
  return n == 0 || memcmp(a.data(), b, sizeof(nnc_job) * n) == 0;
}

#define B_HIP(c, call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      (c)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);           \
      return NNC_E_HIP;                                                             \
    }                                                                               \
  } while (0)

constexpr int kCUs = 256;

// Build the grouped launches (argument tables on the device) for the jobs.
int build_launches(Ctx* c, const std::vector<Net*>& nets, const nnc_job* jobs, int njobs,
                   BatchPlan* plan, std::vector<int>& hsplits, std::vector<int>& hsyms) {
  std::vector<std::vector<PlannedGemm>> per(njobs);
  int maxf = 0, maxr = 0;
  hsplits.assign(njobs, 0);
  hsyms.assign(njobs, 0);
  for (int i = 0; i < njobs; ++i) {
    if (!jobs[i].H || jobs[i].B == 0) continue;
    int rc = internal_plan_tangents(nets[i], jobs[i].B, per[i]);
    if (rc) return rc;
    for (const PlannedGemm& p : per[i]) {
      if (p.phase == 0) maxf = std::max(maxf, p.idx + 1);
      if (p.phase == 1) maxr = std::max(maxr, p.idx + 1);
      if (p.phase == 2) {
        hsplits[i] = p.splits;
        hsyms[i] = p.g.sym;
      }
    }
  }
  const DType ct = nets.empty() ? DT_F32 : nets[0]->ct;
  auto add_launch = [&](int phase, int idx) -> int {
    std::vector<std::pair<GemmArgs, int>> groups;  // (args, splits)
    bool acc64 = false, sym = false;
    long long work = 0;
    for (int i = 0; i < njobs; ++i)
      for (const PlannedGemm& p : per[i])
        if (p.phase == phase && p.idx == idx) {
          groups.push_back({p.g, p.splits});
          acc64 = p.acc64;
          sym = sym || p.g.sym > 0;
          work += (long long)p.g.M * p.g.N * std::max(1, p.g.nbat);
        }
    if (groups.empty()) return NNC_OK;
    // one tiling for the launch: the tuned tiling of its largest product when
    // the table has one the grouped kernel supports, else large tiles when
    // there is work for the chip
    int cfg = work >= (long long)kCUs * 128 * 128 ? 0 : 3;
    {
      const std::pair<GemmArgs, int>* big = &groups[0];
      for (const auto& gr : groups)
        if ((long long)gr.first.M * gr.first.N * gr.first.K > (long long)big->first.M * big->first.N * big->first.K)
          big = &gr;
      auto it = c->tuned.find(TuneKey{(int)ct, big->first.M, big->first.N, big->first.K, (int)acc64, big->second});
      if (it != c->tuned.end() && gemm_grouped_supports(ct, it->second.cfg, acc64)) cfg = it->second.cfg;
    }
    if (!acc64 && c->forced_cfg[ct] >= 0 && gemm_grouped_supports(ct, c->forced_cfg[ct], acc64))
      cfg = c->forced_cfg[ct];
    if (!gemm_grouped_supports(ct, cfg, acc64)) cfg = 3;
    // symmetric layer-sum products need square tiles of their own edge
    // (the 64 x 64 tiling also serves any other H product of the launch)
    if (sym) cfg = kSymCfg;
    long long total = 0;
    std::vector<int> offs(1, 0);
    // cost per tile ~ K / splits: most expensive groups first
    std::sort(groups.begin(), groups.end(), [](const std::pair<GemmArgs, int>& a,
                                               const std::pair<GemmArgs, int>& b) {
      return (long long)a.first.kper < (long long)b.first.kper;
    });
    std::reverse(groups.begin(), groups.end());
    std::vector<GemmArgs> args;
    for (auto& gr : groups) {
      GemmArgs g = gr.first;
      gemm_set_tiles(cfg, g);
      total += (long long)gemm_tiles_per_split(g) * gr.second;
      offs.push_back((int)total);
      args.push_back(g);
    }
    GroupLaunch L;
    L.cfg = cfg;
    L.acc64 = acc64;
    L.ngroups = (int)args.size();
    const int occ = gemm_grouped_occupancy(cfg);
    L.grid = (int)std::min<long long>(total, (long long)kCUs * occ);
    void* a = nullptr;
    void* o = nullptr;
    B_HIP(c, hipMalloc(&a, sizeof(GemmArgs) * args.size()));
    plan->allocs.push_back(a);
    B_HIP(c, hipMalloc(&o, sizeof(int) * offs.size()));
    plan->allocs.push_back(o);
    B_HIP(c, hipMemcpy(a, args.data(), sizeof(GemmArgs) * args.size(), hipMemcpyHostToDevice));
    B_HIP(c, hipMemcpy(o, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice));
    L.dargs = (GemmArgs*)a;
    L.doffs = (int*)o;
    plan->launches.push_back(L);
    return NNC_OK;
  };
  for (int s = 0; s < maxf; ++s) {
    int rc = add_launch(0, s);
    if (rc) return rc;
  }
  for (int r = 0; r < maxr; ++r) {
    int rc = add_launch(1, r);
    if (rc) return rc;
  }
  return add_launch(2, 0);
}

// The captured sequence.
int record(Ctx* c, const std::vector<Net*>& nets, const nnc_job* jobs, int njobs, BatchPlan* plan,
           const std::vector<int>& hsplits, const std::vector<int>& hsyms) {
  for (int i = 0; i < njobs; ++i) {
    const nnc_job& j = jobs[i];
    if (j.B == 0) continue;
    int rc = internal_forward(c, nets[i], j.B, j.x, nullptr, j.g);
    if (!rc && j.J) rc = internal_jacobian(c, nets[i], j.B, j.J);
    if (!rc && j.H) rc = internal_adjoint(c, nets[i], j.B, j.lambda);
    if (!rc && j.H) rc = internal_seed(c, nets[i], j.B);
    if (rc) return rc;
  }
  for (const GroupLaunch& L : plan->launches) {
    ProfRec pr;
    prof_begin(c, NNC_KC_GEMM, &pr);
    B_HIP(c, launch_gemm_grouped(nets[0]->ct, L.cfg, L.acc64, L.dargs, L.doffs, L.ngroups, L.grid,
                                 c->stream));
    prof_end(c, &pr);
  }
  for (int i = 0; i < njobs; ++i) {
    const nnc_job& j = jobs[i];
    if (j.B == 0 || !j.H) continue;
    int rc = internal_softmax_uv(c, nets[i], j.B);
    if (!rc) rc = internal_finalize(c, nets[i], j.B, hsplits[i], j.obj_factor, j.H, hsyms[i]);
    if (rc) return rc;
  }
  return NNC_OK;
}

}  // namespace

void load_tune_cache(Ctx* c) {
  const char* path = getenv("NNC_AUTOTUNE_CACHE");
  if (!path || !path[0]) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    TuneKey k;
    int cfg;
    if (sscanf(line,
               "{\"arch\": \"gfx950\", \"dt\": %d, \"M\": %d, \"N\": %d, \"K\": %d, \"acc64\": %d, "
               "\"splits\": %d, \"cfg\": %d",
               &k.dt, &k.M, &k.N, &k.K, &k.acc64, &k.splits, &cfg) == 7 &&
        cfg >= 0 && cfg < gemm_num_cfgs()) {
      int ks = 1;  // "ksplit" is optional (absent = unsplit)
      const char* q = strstr(line, "\"ksplit\": ");
      if (q) ks = atoi(q + 10);
      if (ks < 1 || ks > 8) ks = 1;
      c->tuned[k] = TuneVal{cfg, ks};
    }
  }
  fclose(f);
}

void free_batch(Ctx* c) {
  BatchState* st = (BatchState*)c->batch;
  if (!st) return;
  free_plan(st->plan);
  if (st->cap) hipStreamDestroy(st->cap);
  delete st;
  c->batch = nullptr;
}

}  // namespace nnc

using namespace nnc;

extern "C" {

int nnc_eval_batch(nnc_ctx ctx, int njobs, const nnc_job* jobs) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (njobs < 0 || (njobs > 0 && !jobs)) {
    c->err = "bad job list";
    return NNC_E_ARG;
  }
  if (njobs == 0) return NNC_OK;
  std::vector<Net*> nets(njobs);
  for (int i = 0; i < njobs; ++i) {
    const nnc_job& j = jobs[i];
    int rc = internal_get_net(c, j.net, &nets[i]);
    if (rc) return rc;
    if (j.B < 0 || j.B > nets[i]->maxB) {
      c->err = "job B outside [0, max_points]";
      return NNC_E_SHAPE;
    }
    if (j.B > 0 && (!j.x || (j.H && !j.lambda))) {
      c->err = "job needs x (and lambda when H is requested)";
      return NNC_E_ARG;
    }
    if (nets[i]->ct != nets[0]->ct) {
      c->err = "all networks of a batch must share one precision";
      return NNC_E_UNSUPPORTED;
    }
    for (int k = 0; k < i; ++k)
      if (jobs[k].net == j.net) {
        c->err = "a network may appear only once per batch (its workspace is per network)";
        return NNC_E_ARG;
      }
  }
  if (hipSetDevice(c->device) != hipSuccess) return NNC_E_HIP;
  BatchState* st = (BatchState*)c->batch;
  if (!st) {
    st = new BatchState();
    c->batch = st;
    B_HIP(c, hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking));
  }
  if (st->plan && same_jobs(st->plan->jobs, njobs, jobs)) {
    ProfRec pr;
    prof_begin(c, NNC_KC_OTHER, &pr);
    B_HIP(c, hipGraphLaunch(st->plan->exec, c->stream));
    prof_end(c, &pr);
    return NNC_OK;
  }
  // (re)plan and capture
  if (st->plan) {
    B_HIP(c, hipStreamSynchronize(c->stream));
    free_plan(st->plan);
    st->plan = nullptr;
  }
  BatchPlan* plan = new BatchPlan();
  plan->jobs.assign(jobs, jobs + njobs);
  std::vector<int> hsplits, hsyms;
  int rc = build_launches(c, nets, jobs, njobs, plan, hsplits, hsyms);
  if (rc) {
    free_plan(plan);
    return rc;
  }
  hipStream_t user = c->stream;
  const bool prof = c->prof;
  const bool dbg = c->debug_checks;
  c->prof = false;
  c->debug_checks = false;
  c->stream = st->cap;
  hipError_t e = hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = record(c, nets, jobs, njobs, plan, hsplits, hsyms);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(st->cap, &g);
    plan->graph = g;
    if (rc == NNC_OK && e2 != hipSuccess) {
      c->err = std::string("graph capture failed: ") + hipGetErrorString(e2);
      rc = NNC_E_HIP;
    }
  } else {
    c->err = std::string("hipStreamBeginCapture failed: ") + hipGetErrorString(e);
    rc = NNC_E_HIP;
  }
  c->stream = user;
  c->prof = prof;
  c->debug_checks = dbg;
  if (rc == NNC_OK) {
    e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      c->err = std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e);
      rc = NNC_E_HIP;
    }
  }
  if (rc) {
    free_plan(plan);
    return rc;
  }
  st->plan = plan;
  ProfRec pr;
  prof_begin(c, NNC_KC_OTHER, &pr);
  B_HIP(c, hipGraphLaunch(plan->exec, c->stream));
  prof_end(c, &pr);
  return NNC_OK;
}

int nnc_autotune(nnc_ctx ctx, int id, int B) {
  Ctx* c = (Ctx*)ctx;
  Net* net;
  int rc = internal_get_net(c, id, &net);
  if (rc) return rc;
  if (B < 1 || B > net->maxB) {
    c->err = "B outside [1, max_points]";
    return NNC_E_SHAPE;
  }
  if (hipSetDevice(c->device) != hipSuccess) return NNC_E_HIP;
  // a captured batch graph was planned with the old tilings (and may hold
  // the old K-split workspace): re-plan on the next batched call
  free_batch(c);
  // synthetic point and multipliers: fill every sweep buffer once
  std::vector<double> hx((size_t)B * net->n, 0.5), hl((size_t)B * net->m, 1.0);
  double* dx = nullptr;
  double* dl = nullptr;
  double* dH = nullptr;
  B_HIP(c, hipMalloc(&dx, hx.size() * 8));
  B_HIP(c, hipMalloc(&dl, hl.size() * 8));
  B_HIP(c, hipMalloc(&dH, (size_t)B * net->n * net->n * 8));
  B_HIP(c, hipMemcpy(dx, hx.data(), hx.size() * 8, hipMemcpyHostToDevice));
  B_HIP(c, hipMemcpy(dl, hl.data(), hl.size() * 8, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  B_HIP(c, hipEventCreate(&e0));
  B_HIP(c, hipEventCreate(&e1));
  const bool prof = c->prof;
  c->prof = false;
  rc = nnc_eval_hess_lag(ctx, id, B, dx, 0.0, dl, dH);
  std::vector<PlannedGemm> plan;
  if (!rc) rc = internal_plan_tangents(net, B, plan);
  FILE* cache = nullptr;
  const char* path = getenv("NNC_AUTOTUNE_CACHE");
  if (!rc && path && path[0]) cache = fopen(path, "a");
  // K-split candidates (FP32 / BF16 sweep GEMMs whose partials stay small):
  // reserve the workspace for the largest one now (plan time)
  constexpr size_t kPartCap = (size_t)256 << 20;  // bytes
  const size_t psz = net->ct == DT_F64 ? 8 : 4;
  // splits 3 and 6 let the last round of workgroups fill the chip where 2
  // and 4 leave it a quarter empty
  const int kKs[] = {2, 3, 4, 6};
  size_t part_need = 0;
  for (const PlannedGemm& p : plan)
    if (internal_ksplit_ok(net, p.g, p.acc64, p.splits))
      for (int ks : kKs)
        if ((size_t)ks * p.g.M * p.g.N * psz <= kPartCap)
          part_need = std::max(part_need, (size_t)ks * p.g.M * p.g.N * psz);
  if (!rc && part_need) rc = internal_ensure_part(c, net, part_need);
  for (size_t pi = 0; !rc && pi < plan.size(); ++pi) {
    PlannedGemm& p = plan[pi];
    if (p.g.sym > 0) continue;  // the symmetric layer-sum product has a fixed tiling
    const TuneKey key{(int)net->ct, p.g.M, p.g.N, p.g.K, (int)p.acc64, p.splits};
    std::vector<int> kss{1};
    if (internal_ksplit_ok(net, p.g, p.acc64, p.splits))
      for (int ks : kKs)
        if ((size_t)ks * p.g.M * p.g.N * psz <= net->part_bytes) kss.push_back(ks);
    struct Trial {
      int cfg, ks;
      float ms;
      double err;  // max |out - reference| / max |reference|
    };
    std::vector<Trial> timed;
    // Validation: every candidate's primary output (out0, M x N at row
    // stride ldo; FP64 for the H products) is compared with that of the
    // plain 64 x 64 register-staged tiling on the same inputs; a candidate
    // further than tol from it is never chosen.
    const DType ot = p.acc64 || p.g.epi == EPI_H64 ? DT_F64 : net->ct;
    const size_t osz = ot == DT_F64 ? 8 : net->csz;
    const size_t ref_elems = (size_t)(p.g.M - 1) * p.g.ldo + p.g.N;
    const double tol = net->ct == DT_BF16 ? 2e-2 : net->ct == DT_F32 ? 1e-4 : 1e-10;
    void* ref = nullptr;
    unsigned* dcmp = nullptr;
    bool have_ref = false;
    if (hipMalloc(&ref, ref_elems * osz) == hipSuccess && hipMalloc(&dcmp, 2 * sizeof(unsigned)) == hipSuccess &&
        gemm_cfg_supports(net->ct, 3, p.acc64)) {
      GemmArgs g = p.g;
      have_ref = internal_launch_gemm_ks(net, g, p.acc64, p.splits, 3, 1, c->stream) == hipSuccess &&
                 hipMemcpyAsync(ref, p.g.out0, ref_elems * osz, hipMemcpyDeviceToDevice, c->stream) == hipSuccess &&
                 hipStreamSynchronize(c->stream) == hipSuccess;
    }
    auto compare = [&]() -> double {  // after a candidate ran: its out0 against the reference
      if (!have_ref) return 0.0;
      unsigned h[2] = {0u, 0u};
      if (hipMemsetAsync(dcmp, 0, 2 * sizeof(unsigned), c->stream) != hipSuccess ||
          launch_max_abs_diff(ot, p.g.out0, ref, p.g.M, p.g.N, p.g.ldo, dcmp, c->stream) != hipSuccess ||
          hipMemcpyAsync(h, dcmp, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
          hipStreamSynchronize(c->stream) != hipSuccess)
        return INFINITY;
      float d, r;
      memcpy(&d, &h[0], 4);
      memcpy(&r, &h[1], 4);
      return (double)d / std::max((double)r, 1e-30);
    };
    int rejected = 0;
    for (int cfg = 0; cfg < gemm_num_cfgs() && !rc; ++cfg) {
      if (!gemm_cfg_supports(net->ct, cfg, p.acc64) || !gemm_cfg_tunable(net->ct, cfg)) continue;
      for (int ks : kss) {
        GemmArgs g = p.g;
        if (internal_launch_gemm_ks(net, g, p.acc64, p.splits, cfg, ks, c->stream) != hipSuccess) continue;
        // two rounds of five launches, the faster round counts (other work on
        // the device shifts single measurements by several percent)
        float ms = 1e30f;
        for (int round = 0; round < 2 && !rc; ++round) {
          hipEventRecord(e0, c->stream);
          const int reps = 5;
          for (int r = 0; r < reps; ++r) internal_launch_gemm_ks(net, g, p.acc64, p.splits, cfg, ks, c->stream);
          hipEventRecord(e1, c->stream);
          if (hipEventSynchronize(e1) != hipSuccess) {
            rc = NNC_E_HIP;
            c->err = "autotune timing failed";
            break;
          }
          float t = 0.f;
          hipEventElapsedTime(&t, e0, e1);
          ms = std::min(ms, t / reps);
        }
        if (rc) break;
        const double err = compare();
        if (err <= tol)
          timed.push_back(Trial{cfg, ks, ms, err});
        else
          ++rejected;
      }
    }
    if (ref) hipFree(ref);
    if (dcmp) hipFree(dcmp);
    if (rc || timed.empty()) break;
    Trial best = timed[0];
    for (const Trial& t : timed)
      if (t.ms < best.ms) best = t;
    // Among choices within 2 % of the fastest (a tie at timing precision),
    // prefer no split, then the largest tile: both re-read less.
    const float best_ms = best.ms;
    for (const Trial& t : timed) {
      if (t.ms > 1.02f * best_ms) continue;
      const long long at = (long long)gemm_cfg(t.cfg).bm * gemm_cfg(t.cfg).bn;
      const long long ab = (long long)gemm_cfg(best.cfg).bm * gemm_cfg(best.cfg).bn;
      if (t.ks < best.ks || (t.ks == best.ks && at > ab)) best = t;
    }
    c->tuned[key] = TuneVal{best.cfg, best.ks};
    if (cache)
      fprintf(cache,
              "{\"arch\": \"gfx950\", \"dt\": %d, \"M\": %d, \"N\": %d, \"K\": %d, \"acc64\": %d, "
              "\"splits\": %d, \"cfg\": %d, \"name\": \"%s\", \"ms\": %.5f, \"ksplit\": %d, "
              "\"validated\": %s, \"max_rel_err\": %.3e, \"candidates\": %d, \"rejected\": %d}\n",
              key.dt, key.M, key.N, key.K, key.acc64, key.splits, best.cfg, gemm_cfg(best.cfg).name, best.ms,
              best.ks, have_ref ? "true" : "false", best.err, (int)timed.size() + rejected, rejected);
  }
  if (cache) fclose(cache);
  c->prof = prof;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(dx);
  hipFree(dl);
  hipFree(dH);
  return rc;
}

int nnc_autotune_query(nnc_ctx ctx, int dtype_prec, int M, int N, int K, int acc64, int splits) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  const int dt = dtype_prec == NNC_FP64 ? DT_F64 : (dtype_prec == NNC_FP32 ? DT_F32 : DT_BF16);
  auto it = c->tuned.find(TuneKey{dt, M, N, K, acc64, splits});
  return it == c->tuned.end() ? -1 : it->second.cfg;
}

}  // extern "C"
