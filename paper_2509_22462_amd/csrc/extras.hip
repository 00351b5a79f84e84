// Batched evaluation, autotuning and warm-start training entry points.
#include "../../include/nnc.h"
#include "nnc_internal.h"

namespace nnc {
void free_trainers(Ctx*) {}
void free_batch(Ctx*) {}
}  // namespace nnc

using namespace nnc;

extern "C" {

int nnc_eval_batch(nnc_ctx ctx, int njobs, const nnc_job* jobs) {
  Ctx* c = (Ctx*)ctx;
  if (!c || (njobs > 0 && !jobs)) return NNC_E_ARG;
  for (int i = 0; i < njobs; ++i) {
    const nnc_job& j = jobs[i];
    if (j.g) {
      int rc = nnc_eval_g(ctx, j.net, j.B, j.x, nullptr, j.g);
      if (rc) return rc;
    }
    if (j.J) {
      int rc = nnc_eval_jac_g(ctx, j.net, j.B, j.x, j.J);
      if (rc) return rc;
    }
    if (j.H) {
      int rc = nnc_eval_hess_lag(ctx, j.net, j.B, j.x, j.obj_factor, j.lambda, j.H);
      if (rc) return rc;
    }
  }
  return NNC_OK;
}

int nnc_autotune(nnc_ctx ctx, int, int) { return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG; }

int nnc_train_create(nnc_ctx ctx, int, const int*, int, int, unsigned long long, int*) {
  return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG;
}
int nnc_train_destroy(nnc_ctx ctx, int) { return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG; }
int nnc_train_step(nnc_ctx ctx, int, const double*, const double*, float, float*) {
  return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG;
}
int nnc_train_predict(nnc_ctx ctx, int, int, const double*, double*) {
  return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG;
}
int nnc_train_num_params(nnc_ctx ctx, int, long long*) { return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG; }
int nnc_train_get_params(nnc_ctx ctx, int, double*) { return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG; }
int nnc_train_set_params(nnc_ctx ctx, int, const double*) { return ctx ? NNC_E_UNSUPPORTED : NNC_E_ARG; }

}  // extern "C"
