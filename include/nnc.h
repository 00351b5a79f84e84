/*
 * nnc.h — C ABI of the MI355X (gfx950) library that evaluates a smooth
 * neural-network constraint y = NN(x) and its derivatives for a
 * reduced-space interior-point method.
 *
 * What it computes (arXiv 2509.22462):
 *   NN(x)      the predictor of Section 3, Eq. 3: z_l = W_l a_{l-1} + b_l,
 *              a_l = sigma_l(z_l), a_0 = x, NN(x) = a_L.
 *   g          the reduced-space constraint residual of Eq. 5 / Section
 *              3.2.1, g(x, y) = y - NN(x)  (or NN(x) itself when y is NULL).
 *   J          the dense Jacobian dNN/dx (m x n), the constraint-Jacobian
 *              oracle of Section 2 (Eq. 2 needs grad g = [-J | I]).
 *   H          the Hessian-of-the-Lagrangian term of Section 3.2.1, Eq. 6:
 *              obj_factor * diag(q) + sum_i lambda_i Hess_x NN_i(x)  (n x n),
 *              computed by differentiating the scalar lambda^T NN(x)
 *              (forward-over-reverse, or the equivalent sum over layers of
 *              T_l^T diag(s_l) T_l), never by forming the m x n x n tensor.
 *   A driver whose constraint is g = y - NN(x) passes lambda_nn = -lambda_g.
 *
 * Conventions for every call:
 *   - Return value: NNC_OK (0) or a negative nnc_status; nothing aborts, no
 *     exception crosses the ABI. nnc_last_error(ctx) describes the failure.
 *   - Caller-owned I/O buffers are contiguous FP64 DEVICE memory (e.g. a
 *     torch.cuda tensor's data_ptr), row-major, unless stated otherwise.
 *   - Calls are asynchronous on the context's HIP stream; the caller
 *     synchronises (or orders later work on the same stream).  A layer-sum
 *     Hessian may run its forward sweep on a second stream that the context
 *     owns (default priority), forked from the context's stream after the
 *     forward pass and joined back to it before the H product, within the
 *     call: every result is still ordered on the context's stream.  The
 *     environment variable NNC_SWEEP_OVERLAP=0 at nnc_create keeps all work
 *     on the context's stream.
 *   - The library allocates device memory only in nnc_create, nnc_net_create
 *     and the nnc_train_* set-up calls — never inside an eval call.
 *   - Results are deterministic: identical inputs give bitwise-identical
 *     outputs (no floating-point atomics; split reductions are summed in a
 *     fixed order).
 *   - Calls on one context must not overlap from several host threads.
 */
#ifndef NNC_H
#define NNC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnc_ctx_s* nnc_ctx;

/* Activation sigma_l per layer. The paper's networks use tanh and sigmoid
 * (Table 1); softplus is the third smooth (C^2) choice Section 2 allows. */
enum nnc_act { NNC_IDENTITY = 0, NNC_TANH = 1, NNC_SIGMOID = 2, NNC_SOFTPLUS = 3, NNC_SOFTMAX = 4 };
/* NNC_SOFTMAX (output layer only; the classifiers of Table 1 end in SoftMax)
 * is not elementwise: NN(x) = softmax(z_L) in FP64, the Jacobian carries
 * dp/dz = diag(p) - p p^T and the Hessian the full second derivative of
 * lambda^T softmax (diag(g) - p g^T - g p^T, g = p * (lambda - p^T lambda)).
 * Networks with a SoftMax output use the layer-sum Hessian method. */

/* Arithmetic of the bulk (tangent/primal/Jacobian) GEMMs. The output-layer
 * reduction forming g and the lambda-weighted adjoint and Hessian
 * accumulation are FP64 in every mode. */
enum nnc_prec { NNC_FP64 = 0, NNC_FP32 = 1, NNC_BF16 = 2 };

enum nnc_status {
  NNC_OK = 0,
  NNC_E_ARG = -1,         /* NULL pointer, bad enum, bad handle            */
  NNC_E_SHAPE = -2,       /* inconsistent dims, B outside [0, max_points]  */
  NNC_E_NOMEM = -3,       /* device allocation failed at set-up            */
  NNC_E_HIP = -4,         /* a HIP runtime call failed                      */
  NNC_E_NONFINITE = -5,   /* NNC_DEBUG_CHECKS set and an input is NaN/Inf  */
  NNC_E_UNSUPPORTED = -6  /* valid request this build does not implement   */
};

/* ------------------------------------------------------------------ context
 * nnc_create: bind device `device` and HIP stream `hip_stream` (a
 * hipStream_t; NULL = the legacy default stream). *out receives the handle.
 * Errors: NNC_E_ARG (out NULL), NNC_E_HIP (bad device). */
int nnc_create(int device, void* hip_stream, nnc_ctx* out);
/* Frees every network, trainer and workspace of the context. NULL is a no-op. */
int nnc_destroy(nnc_ctx ctx);
/* Change the stream later calls are queued on. */
int nnc_set_stream(nnc_ctx ctx, void* hip_stream);
/* Static text for a status code; never NULL. */
const char* nnc_strerror(int status);
/* Text of the last failure on this context ("" if none); owned by ctx. */
const char* nnc_last_error(nnc_ctx ctx);

/* ------------------------------------------------------------------ networks
 * nnc_net_create: register a network of L layers (Section 3, Eq. 3).
 *   dims[0..L]  widths d_0 = n (inputs) ... d_L = m (outputs), all >= 1.
 *   acts[0..L-1] activation of layers 1..L (enum nnc_act). The paper applies
 *               sigma_L at the output too; pass NNC_IDENTITY last for logits.
 *   W[l], b[l]  HOST FP64 arrays of layer l+1: W row-major d_{l+1} x d_l,
 *               b length d_{l+1} (b may be NULL => zero bias). Copied; the
 *               caller keeps ownership and may free them after the call.
 *   prec        enum nnc_prec of the bulk GEMMs.
 *   max_points  largest point count B any eval call on this net will use;
 *               the tangent workspace (about B*n*sum(d_l)*2 elements) is
 *               allocated here.  From 64 points on, calls run the primal
 *               pass and the FP64 adjoint as MFMA GEMMs, so a net created
 *               with max_points >= 64 also holds FP64 copies of its hidden
 *               layers' transposed weights (none extra for NNC_FP64).
 *   *net        receives a handle >= 0.
 * Errors: NNC_E_ARG, NNC_E_SHAPE, NNC_E_NOMEM, NNC_E_HIP. */
int nnc_net_create(nnc_ctx ctx, int L, const int* dims, const int* acts,
                   const double* const* W, const double* const* b, int prec,
                   int max_points, int* net);
int nnc_net_destroy(nnc_ctx ctx, int net);
/* Register the objective diagonal q (DEVICE, FP64, length n, caller-owned,
 * must outlive its use; NULL clears it). eval_hess_lag then adds
 * obj_factor * diag(q) — the sigma * Hess f term of the IPOPT Hessian. */
int nnc_net_set_objective_diag(nnc_ctx ctx, int net, const double* q);
/* Query: dims, precision, max_points; any out pointer may be NULL. */
int nnc_net_info(nnc_ctx ctx, int net, int* L, int* n, int* m, int* prec, int* max_points);

/* Hessian method of eval_hess_lag / nnc_eval / nnc_eval_batch (the same
 * quantity of Section 3.2.1, Eq. 6, by two orders of differentiation):
 *   NNC_HESS_FOR       forward-over-reverse: n forward tangents, then n
 *                      tangents of the lambda-weighted reverse sweep, H = W_1^T G_1;
 *   NNC_HESS_LAYERSUM  z_l is affine in a_{l-1}, so every second-order term
 *                      comes from sigma_l'': H = sum_l T_l^T diag(s_l) T_l with
 *                      T_l = dz_l/dx (the forward tangents) and s_l the FP64
 *                      lambda-weighted adjoint times sigma_l''.  One symmetric
 *                      product over all layers' tangents replaces the reverse
 *                      sweep (cheaper when n is below the hidden widths);
 *   NNC_HESS_AUTO      the cheaper of the two by algorithmic flops for the
 *                      network's shape (chosen at nnc_net_create).
 * nnc_net_set_hess_method may allocate the chosen method's workspace (plan
 * time, never inside an evaluation).  nnc_net_hess_method reports the
 * resolved method (NNC_HESS_FOR or NNC_HESS_LAYERSUM).
 * Errors: NNC_E_ARG (bad handle or method), NNC_E_NOMEM, NNC_E_HIP. */
enum nnc_hess_method { NNC_HESS_AUTO = 0, NNC_HESS_FOR = 1, NNC_HESS_LAYERSUM = 2 };
int nnc_net_set_hess_method(nnc_ctx ctx, int net, int method);
int nnc_net_hess_method(nnc_ctx ctx, int net, int* method);

/* ------------------------------------------------------------------ oracles
 * All three take B points, 0 <= B <= max_points (B = 0 is a no-op).
 *
 * nnc_eval_g: g[b,:] = y[b,:] - NN(x[b,:])   (Eq. 5; g = y - NN(x))
 *   x  DEVICE FP64 [B][n];  y DEVICE FP64 [B][m] or NULL (then g = NN(x));
 *   g  DEVICE FP64 [B][m] (may alias y).  */
int nnc_eval_g(nnc_ctx ctx, int net, int B, const double* x, const double* y, double* g);

/* nnc_eval_g_static: nnc_eval_g for callers that cannot allocate device
 *   memory (code under HIP graph capture, tight serving loops, harnesses
 *   that forbid hipMalloc).  Same arguments, kernels and bits as
 *   nnc_eval_g; the forward pass's per-point vectors (staged input, z_l,
 *   a_l, sigma'_l of every layer) live in a fixed 64 MiB device array that
 *   the library holds on each GPU from load to process exit instead of in
 *   the network's buffers, and the call allocates and frees nothing.  Every
 *   vector is written before it is read, so nothing needs clearing; the
 *   array keeps the last call's contents.  All calls on one GPU share that
 *   array: calls that overlap on one GPU (several streams or host threads)
 *   race and must be serialised by the caller.  The NNC_DEBUG_CHECKS input
 *   scan (a synchronising copy) is not applied.
 * Errors: as nnc_eval_g, plus NNC_E_SHAPE when the B points need more than
 *   64 MiB of vectors (about B * (sum of widths rounded up to 64) * 16 bytes). */
int nnc_eval_g_static(nnc_ctx ctx, int net, int B, const double* x, const double* y, double* g);

/* nnc_eval_jac_g: J[b] = dNN/dx at x[b]  (m x n per point; m batched reverse
 *   passes). x DEVICE FP64 [B][n]; J DEVICE FP64 [B][m][n]. */
int nnc_eval_jac_g(nnc_ctx ctx, int net, int B, const double* x, double* J);

/* nnc_eval_hess_lag: H[b] = obj_factor * diag(q) + sum_i lambda[b,i] Hess NN_i(x[b])
 *   (Section 3.2.1, Eq. 6; n batched forward-over-reverse Hessian-vector
 *   products per point, or the layer sum -- see nnc_net_set_hess_method).
 *   Returned symmetric, in FP64.
 *   x DEVICE FP64 [B][n]; lambda DEVICE FP64 [B][m]; H DEVICE FP64 [B][n][n].
 *   obj_factor is ignored when no objective diagonal is registered. */
int nnc_eval_hess_lag(nnc_ctx ctx, int net, int B, const double* x, double obj_factor,
                      const double* lambda, double* H);

/* nnc_eval: the three oracles above at the same points in one call, sharing
 *   one primal forward pass -- the pattern of an interior-point iteration,
 *   which asks for g, J and the Hessian of the Lagrangian at one x (Section
 *   3.2 and Eq. 2: the Newton system needs all three). Each of g, J, H may be
 *   NULL to skip it (at least one must be given); y is used only with g and
 *   lambda only with H (then required). Outputs are the same bits as the
 *   separate calls. Buffers and shapes as for the separate calls.
 * Errors: NNC_E_ARG (no output, or H without lambda), NNC_E_SHAPE, NNC_E_HIP,
 *   NNC_E_NONFINITE (debug checks). */
int nnc_eval(nnc_ctx ctx, int net, int B, const double* x, const double* y, double obj_factor,
             const double* lambda, double* g, double* J, double* H);

/* ------------------------------------------------------------------ device KKT solve
 * The Newton step of the reduced-space interior-point iteration (Eq. 2 with
 * the barrier terms, after eliminating y, the slack and the multipliers in
 * closed form) is one dense symmetric positive definite system in x per
 * problem.  Solving it next to the Hessian keeps H in HBM (only dx returns
 * to the host); the paper names a GPU-side KKT solver as future work
 * (Section 5.1).  For b < B:
 *     M_b = H_b + diag(d_b) + s_b a_b a_b^T + delta_b I,   M_b dx_b = r_b,
 * by a dense FP64 Cholesky factorisation M_b = L_b L_b^T (blocked,
 * right-looking, 64-column panels) and two triangular solves.
 *
 * nnc_kkt_create: a solver for n x n systems (1 <= n <= 2048), at most max_B
 *   per call; allocates the factor workspace (max_B * n * n doubles) now.
 * nnc_kkt_solve: all pointers DEVICE, FP64 unless noted, caller-owned:
 *   H [B][n][n] (read only; e.g. the output of nnc_eval_hess_lag), d [B][n]
 *   or NULL, a [B][n] and s [B] (both or neither), delta [B] or NULL,
 *   r [B][n]; out: dx [B][n], info [B] (int32): 0 = factorised and solved,
 *   k > 0 = the leading minor of order k of M_b is not positive definite
 *   (LAPACK's convention; dx_b is then 0) -- the caller raises delta_b and
 *   calls again (inertia correction).  Asynchronous on the context's stream.
 * Errors: NNC_E_ARG (bad handle, null pointer, a without s), NNC_E_SHAPE,
 *   NNC_E_NOMEM, NNC_E_HIP. */
int nnc_kkt_create(nnc_ctx ctx, int n, int max_B, int* kkt);
int nnc_kkt_destroy(nnc_ctx ctx, int kkt);
int nnc_kkt_solve(nnc_ctx ctx, int kkt, int B, const double* H, const double* d, const double* a,
                  const double* s, const double* delta, const double* r, double* dx, int* info);

/* nnc_hess_pack_lower: the lower triangle of each symmetric n x n H, row by
 *   row -- the n(n+1)/2 entries of the reduced-space Hessian structure (Table
 *   2 counts them: 307,720 at n = 784), the form in which an interior-point
 *   solver with a sparse-triplet Hessian interface takes it:
 *     Hp[b][i(i+1)/2 + j] = H[b][i][j],  0 <= j <= i < n.
 *   H DEVICE FP64 [B][n][n]; Hp DEVICE FP64 [B][n(n+1)/2], caller-owned, not
 *   aliasing H. Asynchronous on the context's stream; B = 0 is a no-op.
 * Errors: NNC_E_ARG (null or aliasing pointers), NNC_E_SHAPE (B < 0, n < 1). */
int nnc_hess_pack_lower(nnc_ctx ctx, int B, int n, const double* H, double* Hp);

/* ------------------------------------------------------------------ batching
 * One job = one network evaluated at B points (all pointers DEVICE FP64, as
 * for nnc_eval_hess_lag; g and J may be NULL to skip them, H may be NULL). */
typedef struct nnc_job {
  int net;
  int B;
  const double* x;       /* [B][n]    */
  const double* lambda;  /* [B][m]    */
  double obj_factor;
  double* g;             /* [B][m]    NN(x) (no y), or NULL */
  double* J;             /* [B][m][n] or NULL */
  double* H;             /* [B][n][n] or NULL */
} nnc_job;
/* nnc_eval_batch: evaluate several networks at many points in one
 * persistent launch per sweep phase, replayed from a captured HIP graph
 * when the job list matches the previous call's shapes.
 * Errors as for the single-network calls. */
int nnc_eval_batch(nnc_ctx ctx, int njobs, const nnc_job* jobs);

/* nnc_autotune: time every candidate GEMM tiling on each tangent-sweep GEMM
 * shape of this net at B points (synthetic inputs x = 0.5, lambda = 1; HIP
 * events, 3 launches each), keep the fastest per shape in the context's
 * tuning table, and append the choices as JSON lines to the file named by
 * NNC_AUTOTUNE_CACHE when set (read back by nnc_create).  A set-up call: it
 * allocates temporary device buffers and blocks until done; it overwrites
 * the net's sweep workspace (the next eval recomputes everything).
 * nnc_autotune_query: the tuned configuration id of one GEMM shape
 * (dtype = enum nnc_prec), or -1 when the shape is untuned. */
int nnc_autotune(nnc_ctx ctx, int net, int B);
int nnc_autotune_query(nnc_ctx ctx, int prec, int M, int N, int K, int acc64, int splits);
/* nnc_set_gemm_config: force tiling `config` (0 .. nnc_gemm_config_count()-1)
 * for every GEMM of precision `prec` on this context: the tangent sweeps and,
 * from 64 points on, the Jacobian, primal and adjoint products (the
 * FP64-accumulated H product keeps its own choice; a tiling not compiled for
 * that type -- the LDS-DMA tilings for FP64 -- falls back to the heuristic
 * choice; batched launches take it when their grouped kernel supports the
 * tiling, and re-plan on the next nnc_eval_batch); config = -1 restores
 * tuned/heuristic selection.
 * Errors: NNC_E_ARG (unknown config). */
int nnc_set_gemm_config(nnc_ctx ctx, int prec, int config);
int nnc_gemm_config_count(void);
/* nnc_set_gemm_ksplit: run every tangent-sweep GEMM of precision `prec` as
 * `ksplit` K slices (partials -- FP32, or FP64 for FP64 GEMMs -- summed in
 * slice order, then the fused epilogue); 1 = unsplit, -1 restores the tuned
 * choice.  Allocates the partial-sum workspace of the context's networks of
 * that precision now (ksplit * B * n * width elements at B = max_points),
 * never during an evaluation.
 * Errors: NNC_E_ARG (ksplit outside -1, 1..8), NNC_E_NOMEM. */
int nnc_set_gemm_ksplit(nnc_ctx ctx, int prec, int ksplit);

/* ------------------------------------------------------------------ profiling
 * Per-kernel-class timing with HIP events recorded on the context's stream
 * around each launch (the oracle-call breakdown of the paper's Table 4 and
 * the live roofline figures of the benchmark).
 *   nnc_profile(ctx, 1) clears previous records and starts recording;
 *   nnc_profile(ctx, 0) stops.  At most 4096 launches are recorded per
 *   enable; the events are created by nnc_profile(ctx, 1), not by evals.
 *   nnc_profile_read: waits for the recorded work, then returns the summed
 *     duration (ms) and number of launches of one class:
 *       NNC_KC_GEMM     MFMA tangent-sweep GEMMs (forward and reverse sweeps,
 *                       Jacobian rows when B*m >= 64, training GEMMs,
 *                       batched grouped launches)
 *       NNC_KC_SKINNY   weight-streaming kernels (primal, adjoint, Jacobian)
 *       NNC_KC_OTHER    seeds, casts, finalize, graph launches
 *       NNC_KC_GEMM_H   the FP64-accumulated H = G_1 W_1 product
 *   Either out pointer may be NULL. */
enum nnc_kernel_class { NNC_KC_GEMM = 0, NNC_KC_SKINNY = 1, NNC_KC_OTHER = 2, NNC_KC_GEMM_H = 3 };
int nnc_profile(nnc_ctx ctx, int enable);
int nnc_profile_read(nnc_ctx ctx, int kernel_class, double* total_ms, long long* launches);
/* nnc_profile_classes: which kernel classes record events while profiling
 *   is on (bit k = class k; default all, 0xF).  Each recorded launch adds two
 *   event markers to the stream, which cost a few microseconds of queue time
 *   each, so a timed loop records only the class it reports on.
 * Errors: NNC_E_ARG (mask outside 0..0xF). */
int nnc_profile_classes(nnc_ctx ctx, int class_mask);

/* ------------------------------------------------------------------ learned warm start
 * A small MLP (tanh hidden layers, identity output) trained on the GPU with
 * the library's own forward/backward GEMM kernels and an Adam step, used to
 * propose interior-point starting points.
 *   nnc_train_create: dims[0..L], weights initialised N(0, 1/fan_in) from
 *     `seed`, biases 0; `batch` = rows per training step; prec NNC_BF16 or
 *     NNC_FP32 selects the GEMM arithmetic (FP32 master weights always).
 *   nnc_train_step: one Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on
 *     the MSE loss sum((NN(X)-Y)^2)/(batch*d_L); X DEVICE FP64 [batch][d_0],
 *     Y DEVICE FP64 [batch][d_L]; *loss (HOST, may be NULL) receives the loss
 *     before the step (forces a stream synchronisation).
 *   nnc_train_predict: Yhat DEVICE FP64 [B][d_L] for X DEVICE FP64 [B][d_0],
 *     B <= batch.
 *   nnc_train_get/set_params: copy the FP32 master parameters to/from a
 *     HOST FP64 buffer laid out W_1, b_1, W_2, b_2, ... (row-major);
 *     set_params also restarts Adam (moments and step count to zero).
 *   nnc_train_get_grads: the loss gradient of the last nnc_train_step (taken
 *     at the parameters before its update), same HOST layout. */
int nnc_train_create(nnc_ctx ctx, int L, const int* dims, int batch, int prec,
                     unsigned long long seed, int* mlp);
int nnc_train_destroy(nnc_ctx ctx, int mlp);
int nnc_train_step(nnc_ctx ctx, int mlp, const double* X, const double* Y, float lr, float* loss);
int nnc_train_predict(nnc_ctx ctx, int mlp, int B, const double* X, double* Yhat);
int nnc_train_num_params(nnc_ctx ctx, int mlp, long long* count);
int nnc_train_get_params(nnc_ctx ctx, int mlp, double* host_params);
int nnc_train_set_params(nnc_ctx ctx, int mlp, const double* host_params);
int nnc_train_get_grads(nnc_ctx ctx, int mlp, double* host_grads);

/* ------------------------------------------------------------------ peak microbenchmarks
 * The ceilings that the library's kernels are read against, measured on the
 * GPU by plain loops (beside the datasheet peaks): the MFMA-bound tangent
 * sweeps and H products against the matrix-core issue rate, the HBM-bound
 * weight streams (g and J at few points) against the memory stream rate.
 *
 * nnc_peak_mfma: MFMA throughput of one instruction shape (`kind`, below):
 *   16 waves per compute unit, each running 8 independent accumulator
 *   chains of `iters` MFMAs (1 <= iters <= 2^22) from registers; out:
 *   *tflops = executed flops / the launch's event time / 1e12 (HOST double).
 *   Allocates a small result buffer (freed before returning) and waits for
 *   the context's stream.
 * nnc_peak_hbm: stream rate over a caller buffer: src (DEVICE, read only)
 *   and dst (DEVICE, `bytes` long; its contents are overwritten by the copy
 *   and undefined afterwards), both 16-byte aligned and not overlapping,
 *   bytes a positive multiple of 16 (make it well above the 256 MB Infinity
 *   Cache to time HBM); `reps` (1..1000) back-to-back launches are timed.
 *   Out (HOST doubles, either may be NULL but not both): *read_gbs =
 *   bytes read per second / 1e9; *copy_gbs = (bytes read + bytes written)
 *   per second / 1e9.  Waits for the context's stream.
 * Errors: NNC_E_ARG, NNC_E_SHAPE, NNC_E_NOMEM, NNC_E_HIP. */
#define NNC_PEAK_BF16_16X16X32 0 /* v_mfma_f32_16x16x32_bf16 */
#define NNC_PEAK_BF16_32X32X16 1 /* v_mfma_f32_32x32x16_bf16 */
#define NNC_PEAK_FP32_16X16X4 2  /* v_mfma_f32_16x16x4_f32 */
#define NNC_PEAK_FP64_16X16X4 3  /* v_mfma_f64_16x16x4_f64 */
#define NNC_PEAK_NKINDS 4
int nnc_peak_mfma(nnc_ctx ctx, int kind, int iters, double* tflops);
int nnc_peak_hbm(nnc_ctx ctx, const void* src, void* dst, size_t bytes, int reps, double* read_gbs,
                 double* copy_gbs);

#ifdef __cplusplus
}
#endif
#endif /* NNC_H */
