// Warm-start MLP training on the GPU with the library's own kernels.
//
// The network is the MLP of Eq. 3 with tanh hidden layers and an identity
// output, trained by minimising the mean squared error with Adam (the loss
// and optimiser the paper uses for its surrogate networks, Section 4.2).
// Every product is the same MFMA "NT" GEMM as the Hessian sweeps:
//   forward   A_l  = tanh(A_{l-1} W_l^T + b_l)        B operand W_l
//   dgrad     dA   = dZ_l W_l                         B operand W_l^T (copy)
//   wgrad     dW_l = dZ_l^T A_{l-1}                   both operands stored
//                                                     transposed (K = batch)
// with fused epilogues (bias + tanh + sigma', sigma' scaling, transposed
// copies for the next wgrad).  Master parameters and Adam moments are FP32;
// the GEMM copies of W and W^T are BF16 (or FP32).  All reductions are in a
// fixed order, so a step is deterministic.
#include <math.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "../../include/nnc.h"
#include "nnc_device.h"
#include "nnc_internal.h"

namespace nnc {

namespace {

inline int rup(int x, int a) { return (x + a - 1) / a * a; }

struct Trainer {
  int L = 0, batch = 0, bp = 0;
  DType ct = DT_BF16;
  size_t csz = 2;
  std::vector<int> d, dp;
  std::vector<float*> Wm, bm, mW, vW, mb, vb, dW, db;  // per layer (index l-1)
  std::vector<void*> Wc, WTc;
  std::vector<void*> A, AT;     // A[l] l = 0..L-1 (compute type), [bp][dp_l] and [dp_l][bp]
  std::vector<float*> D1;       // sigma' of hidden layers [bp][dp_l]
  std::vector<void*> dZ, dZT;   // per layer l = 1..L
  float* Yhat = nullptr;        // [bp][dp_L]
  double* partial = nullptr;    // loss partial sums
  double* lossd = nullptr;
  int nblocks_loss = 0;
  int step = 0;
  std::vector<void*> allocs;
};

void* talloc(Trainer* t, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) return nullptr;
  if (hipMemset(p, 0, bytes ? bytes : 16) != hipSuccess) {
    hipFree(p);
    return nullptr;
  }
  t->allocs.push_back(p);
  return p;
}

void free_trainer(Trainer* t) {
  if (!t) return;
  for (void* p : t->allocs) hipFree(p);
  delete t;
}

// ---------------------------------------------------------------- kernels
template <typename T>
__global__ void tr_cast_input(const double* X, int rows, int d0, int bp, int dp0, T* A, T* AT) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)bp * dp0) return;
  const int r = (int)(i / dp0);
  const int c = (int)(i % dp0);
  const double v = (r < rows && c < d0) ? X[(long long)r * d0 + c] : 0.0;
  A[i] = from_d<T>(v);
  AT[(long long)c * bp + r] = from_d<T>(v);
}

// dZ_L = 2 (Yhat - Y) / (batch * m) on the true region; per-block loss partials.
template <typename T>
__global__ void tr_mse_grad(const float* Yhat, const double* Y, int batch, int m, int bp, int dpL,
                            T* dZ, T* dZT, double* partial) {
  __shared__ double red[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (i < (long long)bp * dpL) {
    const int r = (int)(i / dpL);
    const int c = (int)(i % dpL);
    float g = 0.f;
    if (r < batch && c < m) {
      const double diff = (double)Yhat[i] - Y[(long long)r * m + c];
      sq = diff * diff;
      g = (float)(2.0 * diff / ((double)batch * m));
    }
    dZ[i] = from_f<T>(g);
    dZT[(long long)c * bp + r] = from_f<T>(g);
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void tr_sum_partials(const double* partial, int n, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// db[j] = sum_k dZT[j][k] in a fixed order.
template <typename T>
__global__ void tr_colsum(const T* dZT, int rows, int bp, float* db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= rows) return;
  float s = 0.f;
  for (int k = 0; k < bp; ++k) s += to_f(dZT[(long long)j * bp + k]);
  db[j] = s;
}

// Adam on one parameter block; refreshes the GEMM copies (W and W^T) when
// `wc` is given.  rows x cols is the padded block shape.
template <typename T>
__global__ void tr_adam(float* p, float* m1, float* m2, const float* g, long long count, int cols,
                        int rows, float lr, float b1, float b2, float eps, float c1, float c2, T* wc,
                        T* wtc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  const float mh = a / c1;
  const float vh = b / c2;
  const float np_ = p[i] - lr * mh / (sqrtf(vh) + eps);
  p[i] = np_;
  if (wc) {
    const int r = (int)(i / cols);
    const int c = (int)(i % cols);
    wc[i] = from_f<T>(np_);
    wtc[(long long)c * rows + r] = from_f<T>(np_);
  }
}

template <typename T>
__global__ void tr_sync(const float* p, long long count, int cols, int rows, T* wc, T* wtc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int r = (int)(i / cols);
  const int c = (int)(i % cols);
  wc[i] = from_f<T>(p[i]);
  wtc[(long long)c * rows + r] = from_f<T>(p[i]);
}

__global__ void tr_out_f64(const float* Yhat, int rows, int m, int dpL, double* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)rows * m) return;
  const int r = (int)(i / m);
  const int c = (int)(i % m);
  out[i] = (double)Yhat[(long long)r * dpL + c];
}

inline unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

#define TR_HIP(c, call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      (c)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);           \
      return NNC_E_HIP;                                                             \
    }                                                                               \
  } while (0)

int get_trainer(Ctx* c, int id, Trainer** out) {
  if (!c) return NNC_E_ARG;
  if (id < 0 || id >= (int)c->trainers.size() || !c->trainers[id]) {
    c->err = "invalid trainer handle";
    return NNC_E_ARG;
  }
  *out = (Trainer*)c->trainers[id];
  return NNC_OK;
}

int tr_gemm(Ctx* c, Trainer* t, GemmArgs g) {
  const long long tiles = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128);
  const int cfg = tiles >= 128 ? 0 : 3;
  g.kper = g.K;
  ProfRec pr;
  prof_begin(c, NNC_KC_GEMM, &pr);
  TR_HIP(c, launch_gemm(t->ct, cfg, false, g, 1, c->stream));
  prof_end(c, &pr);
  return NNC_OK;
}

GemmArgs gargs(const void* A, long long lda, const void* B, long long ldb, int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.lda = lda;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.rdiv = 1;
  return g;
}

template <typename T>
int tr_forward(Ctx* c, Trainer* t, const double* X, int rows) {
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(tr_cast_input<T>, dim3(nblk((long long)t->bp * t->dp[0])), dim3(256), 0, s, X,
                     rows, t->d[0], t->bp, t->dp[0], (T*)t->A[0], (T*)t->AT[0]);
  TR_HIP(c, hipGetLastError());
  for (int l = 1; l <= t->L; ++l) {
    GemmArgs g = gargs(t->A[l - 1], t->dp[l - 1], t->Wc[l - 1], t->dp[l - 1], t->bp, t->dp[l],
                       t->dp[l - 1]);
    g.epi = EPI_TRAIN_FWD;
    g.bias = t->bm[l - 1];
    g.ldo = t->dp[l];
    g.ldt = t->bp;
    if (l < t->L) {
      g.act = ACT_TANH;
      g.out0 = t->A[l];
      g.out1 = t->AT[l];
      g.out2 = t->D1[l];
    } else {
      g.act = ACT_IDENTITY;
      g.out2 = t->Yhat;
    }
    int rc = tr_gemm(c, t, g);
    if (rc) return rc;
  }
  return NNC_OK;
}

template <typename T>
int tr_step(Ctx* c, Trainer* t, const double* X, const double* Y, float lr, float* loss) {
  hipStream_t s = c->stream;
  int rc = tr_forward<T>(c, t, X, t->batch);
  if (rc) return rc;
  const int L = t->L;
  const long long nout = (long long)t->bp * t->dp[L];
  hipLaunchKernelGGL(tr_mse_grad<T>, dim3(nblk(nout)), dim3(256), 0, s, t->Yhat, Y, t->batch,
                     t->d[L], t->bp, t->dp[L], (T*)t->dZ[L], (T*)t->dZT[L], t->partial);
  TR_HIP(c, hipGetLastError());
  hipLaunchKernelGGL(tr_sum_partials, dim3(1), dim3(64), 0, s, t->partial, (int)nblk(nout),
                     1.0 / ((double)t->batch * t->d[L]), t->lossd);
  TR_HIP(c, hipGetLastError());
  for (int l = L; l >= 1; --l) {
    // wgrad: dW_l[dp_l][dp_{l-1}] = dZT_l [dp_l][bp] x AT_{l-1} [dp_{l-1}][bp]^T
    GemmArgs g = gargs(t->dZT[l], t->bp, t->AT[l - 1], t->bp, t->dp[l], t->dp[l - 1], t->bp);
    g.epi = EPI_F32;
    g.out0 = t->dW[l - 1];
    g.ldo = t->dp[l - 1];
    if ((rc = tr_gemm(c, t, g))) return rc;
    hipLaunchKernelGGL(tr_colsum<T>, dim3(nblk(t->dp[l])), dim3(256), 0, s, (const T*)t->dZT[l],
                       t->dp[l], t->bp, t->db[l - 1]);
    TR_HIP(c, hipGetLastError());
    if (l >= 2) {
      // dgrad: dZ_{l-1} = (dZ_l W_l) * sigma'_{l-1};  W_l = (W_l^T)^T
      GemmArgs h = gargs(t->dZ[l], t->dp[l], t->WTc[l - 1], t->dp[l], t->bp, t->dp[l - 1], t->dp[l]);
      h.epi = EPI_TRAIN_BWD;
      h.v0 = t->D1[l - 1];
      h.ldv = t->dp[l - 1];
      h.out0 = t->dZ[l - 1];
      h.out1 = t->dZT[l - 1];
      h.ldo = t->dp[l - 1];
      h.ldt = t->bp;
      if ((rc = tr_gemm(c, t, h))) return rc;
    }
  }
  t->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)t->step);
  const float c2 = 1.f - powf(b2, (float)t->step);
  for (int l = 1; l <= L; ++l) {
    const long long cw = (long long)t->dp[l] * t->dp[l - 1];
    hipLaunchKernelGGL(tr_adam<T>, dim3(nblk(cw)), dim3(256), 0, s, t->Wm[l - 1], t->mW[l - 1],
                       t->vW[l - 1], t->dW[l - 1], cw, t->dp[l - 1], t->dp[l], lr, b1, b2, eps, c1,
                       c2, (T*)t->Wc[l - 1], (T*)t->WTc[l - 1]);
    TR_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(tr_adam<T>, dim3(nblk(t->dp[l])), dim3(256), 0, s, t->bm[l - 1], t->mb[l - 1],
                       t->vb[l - 1], t->db[l - 1], (long long)t->dp[l], t->dp[l], 1, lr, b1, b2, eps,
                       c1, c2, (T*)nullptr, (T*)nullptr);
    TR_HIP(c, hipGetLastError());
  }
  if (loss) {
    double h = 0.0;
    TR_HIP(c, hipMemcpyAsync(&h, t->lossd, sizeof(double), hipMemcpyDeviceToHost, s));
    TR_HIP(c, hipStreamSynchronize(s));
    *loss = (float)h;
  }
  return NNC_OK;
}

template <typename T>
int tr_sync_copies(Ctx* c, Trainer* t) {
  for (int l = 1; l <= t->L; ++l) {
    const long long cw = (long long)t->dp[l] * t->dp[l - 1];
    hipLaunchKernelGGL(tr_sync<T>, dim3(nblk(cw)), dim3(256), 0, c->stream, t->Wm[l - 1], cw,
                       t->dp[l - 1], t->dp[l], (T*)t->Wc[l - 1], (T*)t->WTc[l - 1]);
    TR_HIP(c, hipGetLastError());
  }
  return NNC_OK;
}

int sync_copies(Ctx* c, Trainer* t) {
  return t->ct == DT_BF16 ? tr_sync_copies<bf16>(c, t) : tr_sync_copies<float>(c, t);
}

long long num_params(const Trainer* t) {
  long long n = 0;
  for (int l = 1; l <= t->L; ++l) n += (long long)t->d[l] * t->d[l - 1] + t->d[l];
  return n;
}

}  // namespace

void free_trainers(Ctx* c) {
  for (void* p : c->trainers) free_trainer((Trainer*)p);
  c->trainers.clear();
}

}  // namespace nnc

using namespace nnc;

extern "C" {

int nnc_train_create(nnc_ctx ctx, int L, const int* dims, int batch, int prec,
                     unsigned long long seed, int* mlp) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !dims || !mlp) return NNC_E_ARG;
  if (L < 1 || batch < 1) {
    c->err = "L and batch must be >= 1";
    return NNC_E_SHAPE;
  }
  for (int l = 0; l <= L; ++l)
    if (dims[l] < 1) {
      c->err = "layer widths must be >= 1";
      return NNC_E_SHAPE;
    }
  if (prec != NNC_BF16 && prec != NNC_FP32) {
    c->err = "trainer precision must be NNC_BF16 or NNC_FP32";
    return NNC_E_UNSUPPORTED;
  }
  if (hipSetDevice(c->device) != hipSuccess) return NNC_E_HIP;
  Trainer* t = new Trainer();
  t->L = L;
  t->batch = batch;
  t->bp = rup(batch, 64);
  t->ct = prec == NNC_BF16 ? DT_BF16 : DT_F32;
  t->csz = prec == NNC_BF16 ? 2 : 4;
  for (int l = 0; l <= L; ++l) {
    t->d.push_back(dims[l]);
    t->dp.push_back(rup(dims[l], 64));
  }
  bool ok = true;
  auto A = [&](size_t b) {
    void* p = talloc(t, b);
    if (!p) ok = false;
    return p;
  };
  for (int l = 1; l <= L; ++l) {
    const size_t cw = (size_t)t->dp[l] * t->dp[l - 1];
    t->Wm.push_back((float*)A(cw * 4));
    t->mW.push_back((float*)A(cw * 4));
    t->vW.push_back((float*)A(cw * 4));
    t->dW.push_back((float*)A(cw * 4));
    t->bm.push_back((float*)A(t->dp[l] * 4));
    t->mb.push_back((float*)A(t->dp[l] * 4));
    t->vb.push_back((float*)A(t->dp[l] * 4));
    t->db.push_back((float*)A(t->dp[l] * 4));
    t->Wc.push_back(A(cw * t->csz));
    t->WTc.push_back(A(cw * t->csz));
  }
  t->A.assign(L, nullptr);
  t->AT.assign(L, nullptr);
  t->D1.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    t->A[l] = A((size_t)t->bp * t->dp[l] * t->csz);
    t->AT[l] = A((size_t)t->bp * t->dp[l] * t->csz);
    if (l > 0) t->D1[l] = (float*)A((size_t)t->bp * t->dp[l] * 4);
  }
  t->dZ.assign(L + 1, nullptr);
  t->dZT.assign(L + 1, nullptr);
  for (int l = 1; l <= L; ++l) {
    t->dZ[l] = A((size_t)t->bp * t->dp[l] * t->csz);
    t->dZT[l] = A((size_t)t->bp * t->dp[l] * t->csz);
  }
  t->Yhat = (float*)A((size_t)t->bp * t->dp[L] * 4);
  t->nblocks_loss = (int)nblk((long long)t->bp * t->dp[L]);
  t->partial = (double*)A((size_t)t->nblocks_loss * 8);
  t->lossd = (double*)A(8);
  if (!ok) {
    free_trainer(t);
    c->err = "device allocation failed";
    return NNC_E_NOMEM;
  }
  // N(0, 1/fan_in) initial weights from `seed` (host generator), zero biases.
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (int l = 1; l <= L; ++l) {
    std::vector<float> w((size_t)t->dp[l] * t->dp[l - 1], 0.f);
    const double sc = 1.0 / sqrt((double)dims[l - 1]);
    for (int r = 0; r < dims[l]; ++r)
      for (int q = 0; q < dims[l - 1]; ++q) w[(size_t)r * t->dp[l - 1] + q] = (float)(nd(gen) * sc);
    if (hipMemcpy(t->Wm[l - 1], w.data(), w.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      free_trainer(t);
      c->err = "parameter upload failed";
      return NNC_E_HIP;
    }
  }
  int rc = sync_copies(c, t);
  if (rc == NNC_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = NNC_E_HIP;
  if (rc) {
    free_trainer(t);
    return rc;
  }
  c->trainers.push_back(t);
  *mlp = (int)c->trainers.size() - 1;
  return NNC_OK;
}

int nnc_train_destroy(nnc_ctx ctx, int id) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  hipStreamSynchronize(c->stream);
  free_trainer(t);
  c->trainers[id] = nullptr;
  return NNC_OK;
}

int nnc_train_step(nnc_ctx ctx, int id, const double* X, const double* Y, float lr, float* loss) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (!X || !Y) {
    c->err = "null X or Y";
    return NNC_E_ARG;
  }
  if (hipSetDevice(c->device) != hipSuccess) return NNC_E_HIP;
  return t->ct == DT_BF16 ? tr_step<bf16>(c, t, X, Y, lr, loss) : tr_step<float>(c, t, X, Y, lr, loss);
}

int nnc_train_predict(nnc_ctx ctx, int id, int B, const double* X, double* Yhat) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (B < 0 || B > t->batch) {
    c->err = "B outside [0, batch]";
    return NNC_E_SHAPE;
  }
  if (B == 0) return NNC_OK;
  if (!X || !Yhat) {
    c->err = "null X or Yhat";
    return NNC_E_ARG;
  }
  if (hipSetDevice(c->device) != hipSuccess) return NNC_E_HIP;
  rc = t->ct == DT_BF16 ? tr_forward<bf16>(c, t, X, B) : tr_forward<float>(c, t, X, B);
  if (rc) return rc;
  const int m = t->d[t->L];
  hipLaunchKernelGGL(tr_out_f64, dim3(nblk((long long)B * m)), dim3(256), 0, c->stream, t->Yhat, B, m,
                     t->dp[t->L], Yhat);
  TR_HIP(c, hipGetLastError());
  return NNC_OK;
}

int nnc_train_num_params(nnc_ctx ctx, int id, long long* count) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (!count) return NNC_E_ARG;
  *count = num_params(t);
  return NNC_OK;
}

static int copy_out(Ctx* c, Trainer* t, double* host, bool grads) {
  TR_HIP(c, hipStreamSynchronize(c->stream));
  size_t off = 0;
  for (int l = 1; l <= t->L; ++l) {
    std::vector<float> w((size_t)t->dp[l] * t->dp[l - 1]);
    std::vector<float> b(t->dp[l]);
    TR_HIP(c, hipMemcpy(w.data(), grads ? t->dW[l - 1] : t->Wm[l - 1], w.size() * 4,
                        hipMemcpyDeviceToHost));
    TR_HIP(c, hipMemcpy(b.data(), grads ? t->db[l - 1] : t->bm[l - 1], b.size() * 4,
                        hipMemcpyDeviceToHost));
    for (int r = 0; r < t->d[l]; ++r)
      for (int q = 0; q < t->d[l - 1]; ++q) host[off++] = w[(size_t)r * t->dp[l - 1] + q];
    for (int r = 0; r < t->d[l]; ++r) host[off++] = b[r];
  }
  return NNC_OK;
}

int nnc_train_get_params(nnc_ctx ctx, int id, double* host) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (!host) return NNC_E_ARG;
  return copy_out(c, t, host, false);
}

int nnc_train_get_grads(nnc_ctx ctx, int id, double* host) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (!host) return NNC_E_ARG;
  return copy_out(c, t, host, true);
}

int nnc_train_set_params(nnc_ctx ctx, int id, const double* host) {
  Ctx* c = (Ctx*)ctx;
  Trainer* t;
  int rc = get_trainer(c, id, &t);
  if (rc) return rc;
  if (!host) return NNC_E_ARG;
  TR_HIP(c, hipStreamSynchronize(c->stream));
  size_t off = 0;
  for (int l = 1; l <= t->L; ++l) {
    const size_t cw = (size_t)t->dp[l] * t->dp[l - 1];
    std::vector<float> w(cw, 0.f);
    std::vector<float> b(t->dp[l], 0.f);
    for (int r = 0; r < t->d[l]; ++r)
      for (int q = 0; q < t->d[l - 1]; ++q) w[(size_t)r * t->dp[l - 1] + q] = (float)host[off++];
    for (int r = 0; r < t->d[l]; ++r) b[r] = (float)host[off++];
    TR_HIP(c, hipMemcpy(t->Wm[l - 1], w.data(), cw * 4, hipMemcpyHostToDevice));
    TR_HIP(c, hipMemcpy(t->bm[l - 1], b.data(), b.size() * 4, hipMemcpyHostToDevice));
    // a new parameter set restarts Adam
    TR_HIP(c, hipMemset(t->mW[l - 1], 0, cw * 4));
    TR_HIP(c, hipMemset(t->vW[l - 1], 0, cw * 4));
    TR_HIP(c, hipMemset(t->mb[l - 1], 0, t->dp[l] * 4));
    TR_HIP(c, hipMemset(t->vb[l - 1], 0, t->dp[l] * 4));
  }
  t->step = 0;
  rc = sync_copies(c, t);
  if (rc) return rc;
  TR_HIP(c, hipStreamSynchronize(c->stream));
  return NNC_OK;
}

}  // extern "C"
