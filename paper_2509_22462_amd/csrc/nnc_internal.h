// Internal host-side declarations of libnnc: kernel argument blocks, launch
// entry points and the context / network records behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

namespace nnc {

enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2 };
enum DType { DT_F32 = 0, DT_BF16 = 1, DT_F64 = 2 };

// ---------------------------------------------------------------- MFMA GEMM
// C[M][N] = A[M][K] * B[N][K]^T with both operands K-contiguous ("NT"),
// followed by a fused epilogue.  Rows of A are tangent columns (point b,
// input j) -> row = b * rdiv + j; columns are neurons.
enum GemmEpi {
  EPI_PLAIN = 0,  // out0[row][col] = acc                              (T)
  EPI_FWD_T = 1,  // out0 = acc (T_l), out1 = sigma'[b][col] * acc (P_l)
  EPI_FWD_G = 2,  // out0 = s[b][col] * acc                             (G_last)
  EPI_REV_G = 3,  // out0 = sigma'[b][col]*acc + s[b][col]*aux[row'][col] (G_{l-1})
  EPI_H64 = 4,    // out0 (double) [split][row][col] = acc, FP64 across K tiles
  EPI_JAC_R = 5,  // out0 = acc * sigma'[b][col]  (b = row / rdiv)    (Jacobian rows)
  EPI_F64 = 6,    // out0 (double)[row][col] = acc
  // warm-start MLP training (rows are samples, columns neurons)
  EPI_TRAIN_FWD = 7,  // z = acc + bias[col]; tanh: out0 a, out1 a^T, out2 sigma' (float);
                      // identity: out2 (float) = z
  EPI_TRAIN_BWD = 8,  // dz = acc * v0[row][col] (float); out0 dz, out1 dz^T
  EPI_F32 = 9,        // out0 (float)[row][col] = acc
  EPI_PART = 10,      // out0 (float)[split][row][col] = acc (K-split partial, ld ldo)
  EPI_PART64 = 11,    // out0 (double)[split][row][col] = acc (K-split partial of FP64 GEMMs)
  // primal pass and FP64 adjoint as GEMMs (many points; rows are points)
  EPI_PRIMAL = 12,  // z = acc + bias64[col]: out0 (double) z, out1 (AT) sigma(z), out2 (AT) sigma'(z)
  EPI_ADJ64 = 13,   // FP64 GEMM: out0 = acc * sigma'(z), out1 = acc * sigma''(z), z = v0[row][col]
  // layer-sum Hessian (forward sweep only): out0 = acc (T_l, ld ldo),
  // out2 = s[b][col] * acc (S_l = diag(s_l) T_l, ld ldo), and unless out1 is
  // null out1 = sigma'[b][col] * acc (P_l, the next product's operand, ld ldo1)
  EPI_FWD_LS = 14,
  // the same without S (formed later by scale_layersum_kernel): out0 = T_l,
  // unless out1 is null out1 = P_l
  EPI_FWD_LT = 15,
};

struct GemmArgs {
  const void* A;
  const void* B;
  int M, N, K;
  long long lda, ldb;  // elements
  int kper;            // K elements per split (gridDim.y splits)
  int epi;
  int rdiv;
  void* out0;
  void* out1;
  long long ldo;
  const void* v0;  // sigma' (compute-side type) or s (double), [B][ldv]
  const void* v1;  // s (double) for EPI_REV_G
  long long ldv;
  const void* aux;  // T_{l-1} tile source for EPI_REV_G
  long long ldaux;
  int auxmod;  // aux row = row % auxmod when > 0 (T_1 = W_1^T shared by all points)
  long long split_stride;
  int tiles_m, tiles_n;
  void* out2;         // third output (training epilogues)
  long long ldt;      // leading dimension of transposed outputs
  const float* bias;  // training forward bias
  int act;            // training forward activation; primal / adjoint activation
  const double* bias64;  // EPI_PRIMAL bias
  int dtrue;             // EPI_PRIMAL / EPI_ADJ64: columns >= dtrue are padding (written 0)
  long long ldo1;        // EPI_FWD_LS: row stride of out1
  // Batched products (layer-sum H): nbat > 0 runs nbat independent M x N
  // products; product b reads A from row b * bsA / lda (bsA elements), B
  // from b * bsB, and writes out0 (double) from element b * bsO.  sym > 0:
  // only output tiles on or below the block diagonal (tm >= tn; M == N and
  // BM == BN == sym); the finalize kernel mirrors them.
  int nbat;
  int sym;
  long long bsA, bsB, bsO;
};

// Output tiles of one K split of a product (all its batches).
__host__ __device__ inline int gemm_tiles_per_split(const GemmArgs& g) {
  const int per = g.sym > 0 ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
  return g.nbat > 0 ? g.nbat * per : per;
}

struct GemmCfg {
  int id;
  int bm, bn;
  const char* name;
};
// Tile configurations compiled for each dtype; see gemm.hip.
int gemm_num_cfgs();
const GemmCfg& gemm_cfg(int i);
// acc64: accumulate each K tile's FP32 MFMA result into FP64 registers.
hipError_t launch_gemm(DType t, int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s);
// LDS-DMA-staged tilings (gemm_dma.hip), variant = cfg - kFirstDmaCfg.
constexpr int kFirstDmaCfg = 16;
hipError_t launch_gemm_dma(DType t, int variant, GemmArgs g, int splits, hipStream_t s);
hipError_t launch_gemm_grouped_dma(DType t, int variant, const GemmArgs* groups, const int* offsets, int ngroups,
                                   int grid, hipStream_t s);
int gemm_dma_occupancy(int variant);
// out = epilogue(sum over s of part[s][row][col]) for the epilogue of g
// (partials FP32 for FP32 / BF16 GEMMs, FP64 for FP64; sums in split order).
hipError_t launch_splitk_reduce(DType t, GemmArgs g, const void* part, int splits, hipStream_t s);
bool gemm_cfg_supports(DType t, int cfg, bool acc64);
bool gemm_cfg_tunable(DType t, int cfg);
// Persistent grouped launch over several products (device arrays of GemmArgs
// with tiles_m/tiles_n set, and prefix offsets of work items incl. splits).
bool gemm_grouped_supports(DType t, int cfg, bool acc64);
int gemm_grouped_occupancy(int cfg);
void gemm_set_tiles(int cfg, GemmArgs& g);
hipError_t launch_gemm_grouped(DType t, int cfg, bool acc64, const GemmArgs* groups, const int* offsets,
                               int ngroups, int grid, hipStream_t s);

// ---------------------------------------------------------------- skinny NT
// out[r][j] = sum_k X[r][k] * W[j][k] for few rows r (weight streaming).
enum SkinnyEpi {
  SK_PRIMAL = 0,   // z = acc + bias; out0 z (double), out1 sigma(z), out2 sigma'(z)  (A type)
  SK_JAC_R = 1,    // out0 (A type) = acc * sigma'[r / rdiv][j]
  SK_JAC_OUT = 2,  // out0 (double) = acc
  SK_ADJ = 3,      // abar = acc; out0 zbar = abar*sigma'(z), out1 s = abar*sigma''(z)  (double)
  SK_OUT = 4,      // z = acc + bias; out0 z; out2 sigma'(z) (A); out1 g = y - sigma(z) or sigma(z)
};

struct SkinnyArgs {
  const void* W;
  long long ldw;
  // Optional fragment-packed copy of W (launch_pack_fragments), read by the
  // MFMA stream (5..64 rows) instead of W when set; NULL: row-major W.
  const void* Wp;
  // Optional workspace for K slices across workgroups of the MFMA stream
  // (accumulator type; slice sums of rows x N, or of the adjoint row's N):
  // part_elems elements; NULL: no slicing.
  void* part;
  long long part_elems;
  int N, K;
  const void* X;
  long long ldx;
  int rows;  // rows in this launch (<= template R)
  int row0;  // global index of the first row
  int epi, rdiv, dtrue, act;
  void* out0;
  void* out1;
  void* out2;
  long long ldo;   // out0/out2 row stride (elements)
  long long ldo1;  // out1 row stride
  const double* bias;
  const void* vec;  // z (double) for SK_ADJ, sigma' (A type) for SK_JAC_R
  long long ldv;
  const double* y;  // SK_OUT: residual reference, [B][ldo1] or NULL
};

// S = diag(s_l) T_l for every layer of the layer-sum buffers, after the
// forward sweep wrote T without S (the sweep then needs no adjoint):
// row r = b * n + i of Tc / Sc (ld Ktot), layer l's columns koff[l] ..
// koff[l] + dp[l], s_l = s[l] ([B][dp[l]] doubles).
constexpr int kMaxScaleLayers = 64;
struct LsScaleArgs {
  const void* Tc;
  void* Sc;
  long long ld;
  int rows, n, layers;
  const double* s[kMaxScaleLayers];
  int koff[kMaxScaleLayers];
  int dp[kMaxScaleLayers];
};
hipError_t launch_scale_layersum(DType t, const LsScaleArgs& a, hipStream_t s);

// wt: weight dtype; xt: X dtype; at: accumulator dtype (DT_F32 or DT_F64)
hipError_t launch_skinny(DType wt, DType xt, DType at, SkinnyArgs a, hipStream_t s);
// Fragment-packed copy of W [N][ldw] (K columns, a multiple of 64 / element
// size) for the MFMA weight stream; Wp holds ceil(N/16)*16*K elements.
hipError_t launch_pack_fragments(DType t, const void* W, long long ldw, int N, int K, void* Wp, hipStream_t s);
// One point's Jacobian rows (jac, FP32, 0..64 rows) and FP64 adjoint row
// (adj, 1 row) against the same weights in one stream.
hipError_t launch_reverse_stream(DType wt, SkinnyArgs jac, SkinnyArgs adj, hipStream_t s);

// ---------------------------------------------------------------- elementwise
hipError_t launch_cast_input(DType at, const double* x, int B, int n, void* xin, int np,
                             hipStream_t s);
hipError_t launch_convert_weights(DType t, const double* W, int rows, int cols, void* dst,
                                  int rowsp, int colsp, bool transpose, hipStream_t s);
// P1/G1 seeds: out[b*n + j][k] = W1T[j][k] * vec[b][k]
hipError_t launch_seed_tangent(DType t, const void* W1T, int n, int dp1, const void* vec,
                               bool vec_is_double, int B, void* out, hipStream_t s);
// zbar_L, s_L from lambda and z_L
// (SoftMax output: p [B][mp] holds softmax(z_L); zbar = s = p * (lambda - p^T lambda))
hipError_t launch_adj_seed(const double* lam, const double* zL, int act, int B, int m, int mp,
                           double* zbar, double* sv, const double* p, hipStream_t s);
// SoftMax output layer: p = softmax(z_L) per point (FP64, into p [B][mp],
// padding 0) and g = y - p, or p when y is NULL (g may be NULL).
hipError_t launch_softmax_out(const double* zL, int B, int m, int mp, const double* y, double* g, double* p,
                              hipStream_t s);
// Rank-two part of a SoftMax output's Hessian: u[b][j] = sum_i T[(b,j)][i] p[b][i],
// v[b][j] = sum_i T[(b,j)][i] g[b][i] over the m output columns of the output
// layer's tangents T (compute type, row stride ldt).
hipError_t launch_softmax_uv(DType t, const void* T, long long ldt, int B, int n, int m, int mp, const double* p,
                             const double* g, double* u, double* v, hipStream_t s);
// Jacobian seed rows: R[b*m+i][k] = d1L[b][i] * WL[i][k] * d1prev[b][k]  (d1prev may be NULL)
// (softmax: d1L holds p and the seed is p_i (W_L[i][k] - sum_j p_j W_L[j][k]) d1prev[k])
hipError_t launch_jac_seed(DType at, const double* WL, int m, int K, int Kp, const void* d1L,
                           int ldL, const void* d1prev, int ldp, int B, void* R, bool out_double,
                           bool softmax, hipStream_t s);
// H[b][i][j] = 0.5 * sum_s (P[s][b][i][j] + P[s][b][j][i]) + (i==j) obj * q[i];
// symtile > 0: the partials hold only the tiles on or below the block
// diagonal (edge symtile): below it H[i][j] = sum_s P[s][i][j], above it
// sum_s P[s][j][i], within a diagonal tile the symmetrised sum.
// u, v [B][n] (or NULL): subtract u_i v_j + v_i u_j (a SoftMax output's rank-two term).
hipError_t launch_finalize_h(const double* part, int splits, long long split_stride, int B, int n,
                             double obj, const double* q, double* H, int symtile, const double* u,
                             const double* v, hipStream_t s);
// Layer-sum seeds of layer 1 (T_1 = W_1): for tangent row r = b*n + j and
// column k < dp1, T[r][k] = W1T[j][k], S[r][k] = s_1[b][k] * W1T[j][k]
// (ld ldts), and unless P is null P[r][k] = sigma_1'[b][k] * W1T[j][k] (ld dp1).
hipError_t launch_seed_layersum(DType t, const void* W1T, int n, int dp1, const void* d1, const double* s1,
                                int B, void* T, void* S, long long ldts, void* P, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// Hp[b][i(i+1)/2 + j] = H[b][i][j], j <= i (row-major lower triangle)
hipError_t launch_pack_lower(const double* H, int B, int n, double* Hp, hipStream_t s);
hipError_t launch_check_finite(const double* p, size_t count, int* flag, hipStream_t s);
// out[0] = bits of max |a - ref| (NaN differences count as infinite), out[1]
// = bits of max |ref|, over an M x N matrix of type t (row stride ld); both
// must start at zero.
hipError_t launch_max_abs_diff(DType t, const void* a, const void* ref, int M, int N, long long ld, unsigned* out,
                               hipStream_t s);

// ---------------------------------------------------------------- records
struct Layer {
  int din = 0, dout = 0, dinp = 0, doutp = 0, act = 0;
  void* W = nullptr;   // [doutp][dinp] compute type
  void* WT = nullptr;  // [dinp][doutp] compute type
  void* WTP = nullptr;  // WT packed in the MFMA weight stream's read order (launch_pack_fragments)
  double* b = nullptr;  // [doutp]
  // per-point vectors, [maxB][doutp]
  double* z = nullptr;
  void* a = nullptr;   // A type
  void* d1 = nullptr;  // A type
  double* zbar = nullptr;
  double* s = nullptr;
  // FP64 copy of W^T for the many-point adjoint GEMM (hidden layers of
  // non-FP64 networks created with max_points >= 64; FP64 networks use WT)
  double* WT64 = nullptr;
};

struct Net {
  int L = 0, n = 0, m = 0, np = 0, prec = 0, maxB = 0, Lt = 0;
  DType ct = DT_F32;  // bulk GEMM storage type
  DType at = DT_F32;  // activation / accumulator type
  size_t csz = 4, asz = 4;
  std::vector<Layer> ly;  // ly[l-1] is layer l
  double* WL64 = nullptr;   // output layer [doutp_L][dinp_L], rows >= m zero
  double* WLT64 = nullptr;  // output layer transposed [dinp_L][doutp_L]
  void* xin = nullptr;      // [maxB][np]
  std::vector<void*> P, T;  // tangent buffers indexed by layer (1..Lt-1)
  void* Glast = nullptr;
  // Hessian method: forward-over-reverse (tangent sweeps both ways) or the
  // layer sum H = sum_l T_l^T diag(s_l) T_l (forward sweep, one symmetric
  // product over all layers' tangents)
  int hess_method = 0;  // NNC_HESS_FOR or NNC_HESS_LAYERSUM (resolved, never AUTO)
  bool softmax_out = false;  // SoftMax output layer (layer-sum method only)
  double* usm = nullptr;     // SoftMax rank-two vectors u, v [maxB][n]
  double* vsm = nullptr;
  bool for_bufs = false, ls_bufs = false;  // which method's buffers exist
  void* TC = nullptr;  // layer-sum T_l of all layers, [maxB*n][Ktot], layer l at column koff[l]
  void* SC = nullptr;  // layer-sum S_l = diag(s_l) T_l, same layout
  int Ktot = 0;
  std::vector<int> koff;  // column offset of layer l (1..Lt) in TC / SC
  size_t hpart_bytes = 0;
  double* Hpart = nullptr;
  int hsplit = 1;
  void* part = nullptr;  // K-split partials of the sweep GEMMs (plan-time allocation):
  size_t part_bytes = 0;  // FP32 for FP32/BF16 GEMMs, FP64 for FP64 GEMMs
  void* R0 = nullptr;
  void* R1 = nullptr;
  const double* q = nullptr;
  int* dflag = nullptr;
  // K-slice workspace of the MFMA weight stream (FP32 accumulation):
  // slice sums of <= 64 Jacobian rows and of the adjoint row
  float* spart = nullptr;
  double* spart64 = nullptr;
  long long spart_elems = 0, spart64_elems = 0;
  std::vector<int> tune;  // per-GEMM tuned config (-1 = heuristic)
  std::vector<void*> allocs;
};

struct ProfRec {
  hipEvent_t a, b;
  int kind;
};

// Tuned tiling per GEMM shape: (dtype, M, N, K, acc64, splits) -> config id.
struct TuneKey {
  int dt, M, N, K, acc64, splits;
  bool operator<(const TuneKey& o) const {
    if (dt != o.dt) return dt < o.dt;
    if (M != o.M) return M < o.M;
    if (N != o.N) return N < o.N;
    if (K != o.K) return K < o.K;
    if (acc64 != o.acc64) return acc64 < o.acc64;
    return splits < o.splits;
  }
};

// Tuned choice for a shape: tiling, and (sweep GEMMs only) how many K
// slices to compute as FP32 partials before the fixed-order reduction.
struct TuneVal {
  int cfg = -1;
  int ksplit = 1;
};

struct Ctx {
  int device = 0;
  std::map<TuneKey, TuneVal> tuned;
  int forced_ksplit[3] = {-1, -1, -1};  // per DType, -1 = tuned
  int forced_cfg[3] = {-1, -1, -1};  // per DType
  bool prof = false;
  int prof_mask = 0xF;  // kernel classes recorded while profiling
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<ProfRec> recs;
  hipStream_t stream = nullptr;
  std::string err;
  std::vector<Net*> nets;
  std::vector<void*> trainers;
  bool debug_checks = false;
  void* batch = nullptr;  // batched-evaluation state
  void* scratch = nullptr;  // device address of this device's static workspace (nnc_eval_g_static)
  std::vector<void*> kkts;  // device KKT solvers (kkt.hip)
  // Second stream (default priority) for the layer-sum forward sweep, which
  // runs beside the reverse passes; events fork from and join to `stream`.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> ev_layer;  // forward pass: layer l done (recorded on `stream`)
};

// One GEMM of the tangent sweeps, planned but not launched.
struct PlannedGemm {
  int phase;  // 0 forward-tangent, 1 reverse-tangent, 2 H
  int idx;    // step within the phase
  GemmArgs g;
  bool acc64;
  int splits;
  int slot;  // index in the network's tuning table
};

// Tile edge of the symmetric (lower block triangle) layer-sum H product.
constexpr int kSymTile = 64;
// GEMM tiling id of that product (64 x 64, four waves; FP64-accumulating for
// FP32 and BF16 operands).
constexpr int kSymCfg = 3;

// Internal entry points shared by the runtime, batching, autotuning and
// training modules.
int internal_get_net(Ctx* c, int id, Net** out);
int internal_forward(Ctx* c, Net* net, int B, const double* x, const double* y, double* g);
int internal_jacobian(Ctx* c, Net* net, int B, double* J);
int internal_adjoint(Ctx* c, Net* net, int B, const double* lam);
int internal_tangents(Ctx* c, Net* net, int B, double obj, double* H);
int internal_plan_tangents(Net* net, int B, std::vector<PlannedGemm>& out);
int internal_seed(Ctx* c, Net* net, int B);
hipError_t internal_launch_gemm_ks(Net* net, GemmArgs g, bool acc64, int splits, int cfg, int ks,
                                   hipStream_t s);
bool internal_ksplit_ok(const Net* net, const GemmArgs& g, bool acc64, int splits);
int internal_ensure_part(Ctx* c, Net* net, size_t bytes);
int internal_finalize(Ctx* c, Net* net, int B, int splits, double obj, double* H, int symtile);
// SoftMax output: the rank-two vectors from the output layer's tangents (after the forward sweep).
int internal_softmax_uv(Ctx* c, Net* net, int B);
int internal_pick_cfg(const Net* net, int M, int N, bool acc64);
void free_trainers(Ctx* c);
void free_kkts(Ctx* c);
// Load tuned tilings from the JSON-lines file named by NNC_AUTOTUNE_CACHE.
void load_tune_cache(Ctx* c);
// Profiling brackets around one launch (no-ops unless profiling is on).
int prof_begin(Ctx* c, int kind, ProfRec* r);
void prof_end(Ctx* c, ProfRec* r);
void free_batch(Ctx* c);

}  // namespace nnc
