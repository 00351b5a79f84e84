// Device-resident Newton step of the reduced-space interior-point iteration.
//
// After the closed-form elimination of y, the slack and the multipliers
// (Eq. 2 with the barrier terms), each Newton step is one dense symmetric
// positive definite solve in x:
//     M = H + diag(d) + s a a^T + delta I,      M dx = r,
// with H the Hessian of the Lagrangian that nnc_eval_hess_lag leaves in HBM.
// Solving it on the GPU keeps the n x n Hessian on the device (only dx
// returns to the host), the step the paper names as future work.
//
// Dense Cholesky M = L L^T in FP64, blocked right-looking with 64-column
// panels; B independent systems per call (grid dimension y / x):
//   * kkt_assemble: L = M (full square, row-major), info = 0;
//   * per panel k: kkt_potrf factors the 64 x 64 diagonal block in LDS and
//     writes it back; a pivot that is not positive (or not finite) stops that
//     system with info = its global order (LAPACK's convention: the leading
//     minor of that order is not positive definite); kkt_trsm then solves
//     each 64-row block below against it (L_ik = A_ik L_kk^-T, one row per
//     thread, in LDS);
//   * kkt_update: A_IJ -= L_Ik L_Jk^T on the lower block triangle of the
//     trailing matrix, one 64 x 64 tile per workgroup, 4 x 4 outputs per
//     thread from two panel blocks staged in LDS;
//   * kkt_solve: forward substitution L y = r then back substitution
//     L^T x = y, one workgroup per system: each 64-row block first takes the
//     contributions of the finished blocks (row-contiguous partial dots over
//     16 waves, reduced in a fixed order), then one wave solves the block's
//     triangle from LDS, broadcasting each unknown with a shuffle.
// Every reduction runs in a fixed order: identical inputs give identical bits.
#include <math.h>

#include "../../include/nnc.h"
#include "nnc_device.h"
#include "nnc_internal.h"

namespace nnc {

constexpr int KB = 64;          // panel width
constexpr int kKktMaxN = 2048;  // solve kernel keeps y in LDS

__global__ void kkt_assemble_kernel(const double* __restrict__ H, const double* __restrict__ d,
                                    const double* __restrict__ a, const double* __restrict__ s,
                                    const double* __restrict__ delta, int n, long long total,
                                    double* __restrict__ L, int* __restrict__ info) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const long long nn = (long long)n * n;
  const int b = (int)(t / nn);
  const long long e = t - (long long)b * nn;
  const int i = (int)(e / n);
  const int j = (int)(e - (long long)i * n);
  double v = H[t];
  if (i == j) v += (d ? d[(long long)b * n + i] : 0.0) + (delta ? delta[b] : 0.0);
  if (a && s) v += s[b] * a[(long long)b * n + i] * a[(long long)b * n + j];
  L[t] = v;
  if (e == 0) info[b] = 0;
}

// Factor the w x w lower triangle held in D (LDS) in place; returns 0 or the
// 1-based order of the first pivot that is not positive (all threads).
__device__ int kkt_factor_block(double (*D)[KB + 1], int w, int* s_fail) {
  const int tid = threadIdx.x;
  if (tid == 0) *s_fail = 0;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    if (tid == 0) {
      const double v = D[j][j];
      if (!(v > 0.0) || !isfinite(v))
        *s_fail = j + 1;
      else
        D[j][j] = sqrt(v);
    }
    __syncthreads();
    if (*s_fail) return *s_fail;
    const double ljj = D[j][j];
    for (int i = j + 1 + tid; i < w; i += blockDim.x) D[i][j] /= ljj;
    __syncthreads();
    const int m = w - j - 1;
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      const int i = j + 1 + idx / m;
      const int c = j + 1 + idx % m;
      if (c <= i) D[i][c] -= D[i][j] * D[c][j];
    }
    __syncthreads();
  }
  return 0;
}

// Panel k, diagonal block: factor it in LDS and write L_kk back (lower
// triangle); on a pivot that is not positive record info and stop.
__global__ void __launch_bounds__(256) kkt_potrf_kernel(double* __restrict__ Lall, int n, int k,
                                                        int* __restrict__ info) {
  __shared__ double D[KB][KB + 1];
  __shared__ int s_fail;
  const int b = blockIdx.y;
  if (info[b] != 0) return;
  double* A = Lall + (long long)b * n * n;
  const int kb = k * KB;
  const int w = min(KB, n - kb);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int i = idx / w, j = idx % w;
    D[i][j] = A[(long long)(kb + i) * n + kb + j];
  }
  __syncthreads();
  const int fail = kkt_factor_block(D, w, &s_fail);
  if (fail) {
    if (tid == 0) info[b] = kb + fail;
    return;
  }
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int i = idx / w, j = idx % w;
    if (j <= i) A[(long long)(kb + i) * n + kb + j] = D[i][j];
  }
}

// Panel k, row block k + 1 + blockIdx.x: L_ik = A_ik L_kk^-T, one row per
// thread, the factored diagonal block and the row block staged in LDS.
__global__ void __launch_bounds__(256) kkt_trsm_kernel(double* __restrict__ Lall, int n, int k,
                                                       const int* __restrict__ info) {
  __shared__ double D[KB][KB + 1];
  __shared__ double R[KB][KB + 1];
  const int b = blockIdx.y;
  if (info[b] != 0) return;
  double* A = Lall + (long long)b * n * n;
  const int kb = k * KB;
  const int w = min(KB, n - kb);
  const int r0 = (k + 1 + blockIdx.x) * KB;
  const int nr = min(KB, n - r0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < w * w; idx += blockDim.x) {
    const int i = idx / w, j = idx % w;
    D[i][j] = j <= i ? A[(long long)(kb + i) * n + kb + j] : 0.0;
  }
  for (int idx = tid; idx < nr * w; idx += blockDim.x) {
    const int i = idx / w, j = idx % w;
    R[i][j] = A[(long long)(r0 + i) * n + kb + j];
  }
  __syncthreads();
  // row i of the block: x_j = (a_j - sum_{t<j} x_t L_kk[j][t]) / L_kk[j][j]
  for (int i = tid; i < nr; i += blockDim.x) {
    for (int j = 0; j < w; ++j) {
      double v = R[i][j];
      for (int t = 0; t < j; ++t) v -= R[i][t] * D[j][t];
      R[i][j] = v / D[j][j];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nr * w; idx += blockDim.x) {
    const int i = idx / w, j = idx % w;
    A[(long long)(r0 + i) * n + kb + j] = R[i][j];
  }
}

// Trailing update after panel k: tile (I, J), I >= J > k, of the lower block
// triangle, enumerated row by row.
__global__ void __launch_bounds__(256) kkt_update_kernel(double* __restrict__ Lall, int n, int k,
                                                         const int* __restrict__ info) {
  __shared__ double LI[KB][KB + 1];
  __shared__ double LJ[KB][KB + 1];
  const int b = blockIdx.y;
  if (info[b] != 0) return;
  double* A = Lall + (long long)b * n * n;
  int t = blockIdx.x;
  int ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (ti > 0 && ti * (ti + 1) / 2 > t) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int tj = t - ti * (ti + 1) / 2;
  const int I0 = (k + 1 + ti) * KB, J0 = (k + 1 + tj) * KB;
  const int kb = k * KB;
  const int w = min(KB, n - kb);
  const int ni = min(KB, n - I0), nj = min(KB, n - J0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < KB * KB; idx += blockDim.x) {
    const int r = idx / KB, c = idx % KB;
    LI[r][c] = (r < ni && c < w) ? A[(long long)(I0 + r) * n + kb + c] : 0.0;
    LJ[r][c] = (r < nj && c < w) ? A[(long long)(J0 + r) * n + kb + c] : 0.0;
  }
  __syncthreads();
  const int ty = tid >> 4, tx = tid & 15;
  double acc[4][4] = {};
  for (int c = 0; c < w; ++c) {
    double li[4], lj[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      li[u] = LI[ty * 4 + u][c];
      lj[u] = LJ[tx * 4 + u][c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = fma(li[u], lj[v], acc[u][v]);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ty * 4 + u, c = tx * 4 + v;
      if (r < ni && c < nj) A[(long long)(I0 + r) * n + J0 + c] -= acc[u][v];
    }
}

// Forward and back substitution with the factor L (lower triangle of each
// system's matrix); 1024 threads = 16 waves per system.
__global__ void __launch_bounds__(1024) kkt_solve_kernel(const double* __restrict__ Lall, int n,
                                                         const double* __restrict__ r, double* __restrict__ x,
                                                         const int* __restrict__ info) {
  __shared__ double y[kKktMaxN];
  __shared__ double D[KB][KB + 1];
  __shared__ double part[16][KB];
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  if (info[b] != 0) {
    for (int i = tid; i < n; i += blockDim.x) x[(long long)b * n + i] = 0.0;
    return;
  }
  const double* L = Lall + (long long)b * n * n;
  for (int i = tid; i < n; i += blockDim.x) y[i] = r[(long long)b * n + i];
  __syncthreads();
  const int nblk = (n + KB - 1) / KB;
  // forward: L y = r
  for (int k = 0; k < nblk; ++k) {
    const int kb = k * KB, w = min(KB, n - kb);
    // contributions of the finished unknowns y[0..kb) to rows kb..kb+w
    for (int i = wv; i < w; i += 16) {
      const double* row = L + (long long)(kb + i) * n;
      double sacc = 0.0;
      for (int t = lane; t < kb; t += 64) sacc += row[t] * y[t];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
      if (lane == 0) part[0][i] = sacc;
    }
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = idx / w, j = idx % w;
      D[i][j] = j <= i ? L[(long long)(kb + i) * n + kb + j] : 0.0;
    }
    __syncthreads();
    if (wv == 0) {
      double yi = lane < w ? y[kb + lane] - part[0][lane] : 0.0;
      for (int j = 0; j < w; ++j) {
        const double yj = __shfl(yi / D[j][j], j, 64);
        if (lane == j) yi = yj;
        if (lane > j && lane < w) yi -= D[lane][j] * yj;
      }
      if (lane < w) y[kb + lane] = yi;
    }
    __syncthreads();
  }
  // back: L^T x = y (x overwrites y)
  for (int k = nblk - 1; k >= 0; --k) {
    const int kb = k * KB, w = min(KB, n - kb);
    // contributions of the finished unknowns x[kb+w..n) to rows kb..kb+w of
    // L^T: sum over t of L[t][kb+i] x[t]; wave wv takes rows t = kb+w+wv+16q
    double sacc = 0.0;
    if (lane < w)
      for (int t = kb + w + wv; t < n; t += 16) sacc += L[(long long)t * n + kb + lane] * y[t];
    part[wv][lane] = sacc;
    for (int idx = tid; idx < w * w; idx += blockDim.x) {
      const int i = idx / w, j = idx % w;
      D[i][j] = j <= i ? L[(long long)(kb + i) * n + kb + j] : 0.0;
    }
    __syncthreads();
    if (wv == 0) {
      double tot = 0.0;
      for (int q = 0; q < 16; ++q) tot += part[q][lane];
      double xi = lane < w ? y[kb + lane] - tot : 0.0;
      for (int i = w - 1; i >= 0; --i) {
        const double xv = __shfl(xi / D[i][i], i, 64);
        if (lane == i) xi = xv;
        if (lane < i) xi -= D[i][lane] * xv;
      }
      if (lane < w) y[kb + lane] = xi;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += blockDim.x) x[(long long)b * n + i] = y[i];
}

struct Kkt {
  int n = 0, maxB = 0;
  double* L = nullptr;
};

void free_kkts(Ctx* c) {
  for (void* p : c->kkts) {
    Kkt* k = (Kkt*)p;
    if (!k) continue;
    hipFree(k->L);
    delete k;
  }
  c->kkts.clear();
}

}  // namespace nnc

using namespace nnc;

namespace {
int kkt_fail(Ctx* c, int code, const char* msg) {
  if (c) c->err = msg;
  return code;
}
}  // namespace

extern "C" {

int nnc_kkt_create(nnc_ctx ctx, int n, int max_B, int* kkt) {
  Ctx* c = (Ctx*)ctx;
  if (!c || !kkt) return kkt_fail(c, NNC_E_ARG, "null argument");
  if (n < 1 || n > kKktMaxN || max_B < 1) return kkt_fail(c, NNC_E_SHAPE, "n outside 1..2048 or max_B < 1");
  if (hipSetDevice(c->device) != hipSuccess) return kkt_fail(c, NNC_E_HIP, "hipSetDevice failed");
  Kkt* k = new Kkt();
  k->n = n;
  k->maxB = max_B;
  if (hipMalloc(&k->L, (size_t)max_B * n * n * sizeof(double)) != hipSuccess) {
    delete k;
    return kkt_fail(c, NNC_E_NOMEM, "KKT factor workspace");
  }
  c->kkts.push_back(k);
  *kkt = (int)c->kkts.size() - 1;
  return NNC_OK;
}

int nnc_kkt_destroy(nnc_ctx ctx, int kkt) {
  Ctx* c = (Ctx*)ctx;
  if (!c || kkt < 0 || kkt >= (int)c->kkts.size() || !c->kkts[kkt]) return kkt_fail(c, NNC_E_ARG, "invalid KKT handle");
  Kkt* k = (Kkt*)c->kkts[kkt];
  hipStreamSynchronize(c->stream);
  hipFree(k->L);
  delete k;
  c->kkts[kkt] = nullptr;
  return NNC_OK;
}

int nnc_kkt_solve(nnc_ctx ctx, int kkt, int B, const double* H, const double* d, const double* a, const double* s,
                  const double* delta, const double* r, double* dx, int* info) {
  Ctx* c = (Ctx*)ctx;
  if (!c || kkt < 0 || kkt >= (int)c->kkts.size() || !c->kkts[kkt]) return kkt_fail(c, NNC_E_ARG, "invalid KKT handle");
  Kkt* k = (Kkt*)c->kkts[kkt];
  if (B < 0 || B > k->maxB) return kkt_fail(c, NNC_E_SHAPE, "B outside [0, max_B]");
  if (B == 0) return NNC_OK;
  if (!H || !r || !dx || !info) return kkt_fail(c, NNC_E_ARG, "null H, r, dx or info");
  if ((a == nullptr) != (s == nullptr)) return kkt_fail(c, NNC_E_ARG, "a and s must be given together");
  if (hipSetDevice(c->device) != hipSuccess) return kkt_fail(c, NNC_E_HIP, "hipSetDevice failed");
  const int n = k->n;
  const long long total = (long long)B * n * n;
  const long long blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffLL) return kkt_fail(c, NNC_E_SHAPE, "B * n * n too large");
  ProfRec pr;
  prof_begin(c, NNC_KC_OTHER, &pr);
  hipLaunchKernelGGL(kkt_assemble_kernel, dim3((unsigned)blocks), dim3(256), 0, c->stream, H, d, a, s, delta, n,
                     total, k->L, info);
  const int nblk = (n + KB - 1) / KB;
  for (int p = 0; p < nblk; ++p) {
    hipLaunchKernelGGL(kkt_potrf_kernel, dim3(1, B), dim3(256), 0, c->stream, k->L, n, p, info);
    const int T = nblk - p - 1;
    if (T == 0) break;
    hipLaunchKernelGGL(kkt_trsm_kernel, dim3(T, B), dim3(256), 0, c->stream, k->L, n, p, (const int*)info);
    hipLaunchKernelGGL(kkt_update_kernel, dim3(T * (T + 1) / 2, B), dim3(256), 0, c->stream, k->L, n, p,
                       (const int*)info);
  }
  hipLaunchKernelGGL(kkt_solve_kernel, dim3(B), dim3(1024), 0, c->stream, (const double*)k->L, n, r, dx,
                     (const int*)info);
  const hipError_t e = hipGetLastError();
  prof_end(c, &pr);
  if (e != hipSuccess) {
    c->err = std::string("KKT kernels: ") + hipGetErrorString(e);
    return NNC_E_HIP;
  }
  return NNC_OK;
}

}  // extern "C"
