// Weight-streaming kernels for the few-row products of the method, plus the
// small elementwise kernels around the GEMMs.
//
// skinny_ksplit_kernel computes out[r][j] = sum_k X[r][k] * W[j][k] for at
// most 4 rows r (points); skinny_mfma_kernel and skinny_rows_lds_kernel
// below take 5..64 rows (Jacobian rows b*m+i, optionally with one FP64
// adjoint row).  These
// products are bound by HBM bandwidth (each weight is used 2R times), so the
// kernels stream W once with full 16-byte coalesced loads, keep several KiB
// of the stream in flight per wave, and split K across the waves of a
// workgroup so that a launch has thousands of waves.  The R rows of X are
// re-read from L1/L2 (they are tiny and shared by all waves of the CU).
// Each (row, j) result goes through the fused epilogue: bias and
// sigma/sigma'/sigma'' for the primal pass, sigma' scaling for Jacobian rows,
// sigma'/sigma'' products for the FP64 adjoint, the FP64 residual.
#include <algorithm>
#include <type_traits>

#include "nnc_device.h"
#include "nnc_internal.h"

namespace nnc {

template <typename TX, typename A, int WV>
__device__ __forceinline__ void load_x(const TX* p, A* o) {
  constexpr int BYTES = (int)sizeof(TX) * WV;
  if constexpr (BYTES >= 16) {
    constexpr int NV = BYTES / 16;
    constexpr int PER = 16 / (int)sizeof(TX);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const uint4 u = ((const uint4*)p)[v];
      Vec16<TX, A>::unpack(u, o + v * PER);
    }
  } else {
    static_assert(BYTES == 8, "unsupported X vector");
    const uint2 u = *(const uint2*)p;
    o[0] = (A)__uint_as_float(u.x);
    o[1] = (A)__uint_as_float(u.y);
  }
}

template <typename A> __device__ __forceinline__ A wave_sum(A v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename A>
__device__ __forceinline__ void skinny_epilogue(const SkinnyArgs& a, int row, int j, A v) {
  const long long o = (long long)row * a.ldo + j;
  switch (a.epi) {
    case SK_PRIMAL: {
      double z = 0.0;
      ActVal av{0.0, 0.0, 0.0};
      if (j < a.dtrue) {
        z = (double)v + a.bias[j];
        av = act_eval(a.act, z);
      }
      ((double*)a.out0)[o] = z;
      ((A*)a.out1)[o] = (A)av.v;
      ((A*)a.out2)[o] = (A)av.d1;
      break;
    }
    case SK_JAC_R: {
      const int b = row / a.rdiv;
      const A d1 = ((const A*)a.vec)[(long long)b * a.ldv + j];
      ((A*)a.out0)[o] = v * d1;
      break;
    }
    case SK_JAC_OUT:
      ((double*)a.out0)[o] = (double)v;
      break;
    case SK_ADJ: {
      double zb = 0.0, sv = 0.0;
      if (j < a.dtrue) {
        const double z = ((const double*)a.vec)[(long long)row * a.ldv + j];
        const ActVal av = act_eval(a.act, z);
        zb = (double)v * av.d1;
        sv = (double)v * av.d2;
      }
      ((double*)a.out0)[o] = zb;
      ((double*)a.out1)[(long long)row * a.ldo1 + j] = sv;
      break;
    }
    case SK_OUT: {
      const double z = (double)v + a.bias[j];
      const ActVal av = act_eval(a.act, z);
      ((double*)a.out0)[o] = z;
      ((double*)a.out2)[o] = av.d1;
      if (a.out1) {
        const long long go = (long long)row * a.ldo1 + j;
        ((double*)a.out1)[go] = a.y ? a.y[go] - av.v : av.v;
      }
      break;
    }
  }
}

// FMA weight stream for at most 4 rows: a workgroup of KSPLIT waves owns JR
// consecutive weight rows and its waves split K, so a launch has
// (N / JR) * KSPLIT waves -- enough independent loads in flight to cover
// HBM latency even though each wave waits for its own loads every U
// vectors.  Lanes walk K in 16-byte vectors (one load instruction moves a
// contiguous KiB of a row); U vectors per row are loaded before any is
// used; the R rows of X are re-read from L1/L2.  Per-wave partial sums are
// reduced across the wave with shuffles, then across the waves in LDS in
// wave order (fixed order, deterministic), and one thread per (row, j)
// applies the fused epilogue.
template <typename TW, typename TX, typename A, int R, int JR, int KSPLIT>
__global__ void __launch_bounds__(KSPLIT * 64) skinny_ksplit_kernel(SkinnyArgs a) {
  constexpr int WV = 16 / (int)sizeof(TW);
  constexpr int U = R <= 2 ? 4 : 2;
  __shared__ A red[KSPLIT][JR * R];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * JR;
  const int nvec = a.K / WV;  // K is a multiple of WV
  const int per = ((nvec + KSPLIT - 1) / KSPLIT + 63) / 64 * 64;
  const int v0 = wave * per;
  const int v1 = min(nvec, v0 + per);
  A acc[JR][R];
#pragma unroll
  for (int q = 0; q < JR; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[q][r] = (A)0;
  const TW* W = (const TW*)a.W;
  const TX* X = (const TX*)a.X;
  const TW* wrow[JR];
#pragma unroll
  for (int q = 0; q < JR; ++q) wrow[q] = W + (long long)min(j0 + q, a.N - 1) * a.ldw;
  for (int vb = v0 + lane; vb < v1; vb += 64 * U) {
    uint4 u[U][JR];
#pragma unroll
    for (int v = 0; v < U; ++v)
#pragma unroll
      for (int q = 0; q < JR; ++q) {
        const int vv = vb + v * 64;
        u[v][q] = (vv < v1 && j0 + q < a.N) ? *(const uint4*)(wrow[q] + (long long)vv * WV)
                                             : make_uint4(0u, 0u, 0u, 0u);
      }
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const int vv = vb + v * 64;
      if (vv < v1) {
        const int k = vv * WV;
        A w[JR][WV];
#pragma unroll
        for (int q = 0; q < JR; ++q) Vec16<TW, A>::unpack(u[v][q], w[q]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (r < a.rows) {
            A xv[WV];
            load_x<TX, A, WV>(X + (long long)r * a.ldx + k, xv);
#pragma unroll
            for (int q = 0; q < JR; ++q)
#pragma unroll
              for (int e = 0; e < WV; ++e) acc[q][r] += w[q][e] * xv[e];
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < JR; ++q)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const A t = wave_sum(acc[q][r]);
      if (lane == 0) red[wave][q * R + r] = t;
    }
  __syncthreads();
  if (threadIdx.x < JR * R) {
    const int q = threadIdx.x / R;
    const int r = threadIdx.x % R;
    A v = red[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < KSPLIT; ++w) v += red[w][threadIdx.x];
    if (j0 + q < a.N && r < a.rows) skinny_epilogue<A>(a, a.row0 + r, j0 + q, v);
  }
}

// MFMA form of the weight stream, for more than 4 rows (Jacobian rows): a
// workgroup of KSPLIT waves owns 16 weight rows j0..j0+15 and the waves split
// K.  Per step each lane loads 16 bytes of one weight row (lane % 16) and the
// matching K range of one X row (lane % 16; rows >= `rows` read as 0) and
// issues one 16x16x4 MFMA per element, D[r][j] += X[r][k] W[j][k]: up to 16
// X rows ride in the A operand, so X is re-read once per weight byte rather
// than once per row.  Partial blocks are summed in LDS in wave order.
template <typename A> struct SkMma;
template <> struct SkMma<float> {
  using Acc = floatx4;
  __device__ __forceinline__ static Acc mma(float x, float w, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, w, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int e) { return (lane >> 4) * 4 + e; }
};
template <> struct SkMma<double> {
  using Acc = doublex4;
  __device__ __forceinline__ static Acc mma(double x, double w, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, w, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};

// RB row blocks of 16 X rows (up to 64 Jacobian rows) share each weight
// fragment: one read of the weights serves every row, and the RB
// accumulators (two per block, even and odd elements, so consecutive MFMAs
// never wait on each other's result) are independent chains.
//
// With ADJ the same weight stream also carries the FP64 adjoint row of one
// point (d: X = zbar_l in FP64, epilogue SK_ADJ): the Jacobian rows and the
// adjoint both multiply by W_l^T in reverse layer order, so one read of the
// weights serves both.  Each lane adds its weights times the adjoint entries
// of its K range in FP64 (two partial sums, even and odd elements); the
// partial dots are reduced over the four lane groups by shuffles and over the
// waves in LDS, in a fixed order.  JAC = false streams the adjoint alone
// through the same code (same rounding).
//
// PACKED: the weights come from a.Wp, a copy stored in the order the lanes
// read it (pack_fragments_kernel): for 16-row block jb and K step s, the 64
// lanes' 16-byte chunks are one contiguous KiB, so each wave load moves a
// whole KiB instead of 64 bytes from each of 16 rows.  Same elements, same
// order, same results.
template <typename TW, typename TX, typename A, int KSPLIT, int RB, bool JAC = true, bool ADJ = false,
          bool PACKED = false, int NB = 1>
__global__ void __launch_bounds__(KSPLIT * 64) skinny_mfma_kernel(SkinnyArgs a, SkinnyArgs d) {
  using M = SkMma<A>;
  constexpr int WV = 16 / (int)sizeof(TW);  // weight elements per 16-byte load
  constexpr int KSTEP = 4 * WV;             // K covered by one wave step
  constexpr int NR = JAC ? 16 * RB : 1;     // X rows carried (multiple of 16)
  constexpr bool BF16_MMA = sizeof(TW) == 2 && sizeof(A) == 4;  // BF16 weights, FP32 rows
  __shared__ A red[JAC ? NB * KSPLIT : 1][NR][17];
  __shared__ double red_adj[ADJ ? NB * KSPLIT : 1][16];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int j0 = blockIdx.x * 16 * NB;  // NB blocks of 16 weight rows per workgroup
  const int c16 = lane & 15;
  const int q = lane >> 4;
  const int nsteps = a.K / KSTEP;
  // K slices across workgroups (gridDim.y > 1): slice blockIdx.y of the K
  // steps, split over the waves; the slices' sums go to a.part / d.part and
  // a reduction in slice order applies the epilogue
  const int kslices = gridDim.y;
  const int sper = (nsteps + kslices - 1) / kslices;
  const int ws0 = min(nsteps, (int)blockIdx.y * sper);
  const int ws1 = min(nsteps, ws0 + sper);
  const int per = (ws1 - ws0 + KSPLIT - 1) / KSPLIT;
  const int s0 = min(ws1, ws0 + wave * per);
  const int s1 = min(ws1, s0 + per);
  // element offset of this lane's chunk of block nb at step s: wp[nb] + s * wstep
  bool wok[NB];
  const TW* wp[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int j = j0 + nb * 16 + c16;
    // packed copies hold whole 16-row blocks (zero rows past N); a block
    // past the last one is skipped
    wok[nb] = PACKED ? j0 + nb * 16 < a.N : j < a.N;
    wp[nb] = PACKED ? (const TW*)a.Wp + (((long long)blockIdx.x * NB + nb) * nsteps * 64 + lane) * WV
                    : (const TW*)a.W + (long long)(wok[nb] ? j : 0) * a.ldw + q * WV;
  }
  constexpr long long wstep = PACKED ? 64 * WV : KSTEP;
  const TX* xp[RB];
  bool xok[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    xok[rb] = JAC && rb * 16 + c16 < a.rows;
    xp[rb] = (const TX*)a.X + (long long)(xok[rb] ? rb * 16 + c16 : 0) * a.ldx + q * WV;
  }
  const double* dp = ADJ ? (const double*)d.X + q * WV : nullptr;
  typename M::Acc acc[NB][RB][2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[nb][rb][0] = acc[nb][rb][1] = typename M::Acc{0, 0, 0, 0};
  double adj[NB][2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) adj[nb][0] = adj[nb][1] = 0.0;
  // U steps of W and X are loaded before the MFMAs that use them, keeping
  // U KiB of the weight stream per block in flight per wave (U changes no
  // rounding: the steps are accumulated in order either way).  Each X (and
  // adjoint) fragment serves the NB weight blocks.
  constexpr int U = NB > 1 ? 2 : ((ADJ && WV == 8) || RB > 2 ? 2 : 4);
  for (int sb = s0; sb < s1; sb += U) {
    uint4 wu[U][NB];
    A xf[JAC ? U : 1][RB][WV];
    double xd[ADJ ? U : 1][WV];
#pragma unroll
    for (int v = 0; v < U; ++v) {
      const bool in = sb + v < s1;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        wu[v][nb] = (wok[nb] && in) ? *(const uint4*)(wp[nb] + (long long)(sb + v) * wstep)
                                    : make_uint4(0u, 0u, 0u, 0u);
      const int k = (sb + v) * KSTEP;
      if constexpr (JAC) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if (xok[rb] && in) {
            load_x<TX, A, WV>(xp[rb] + k, xf[v][rb]);
          } else {
#pragma unroll
            for (int e = 0; e < WV; ++e) xf[v][rb][e] = (A)0;
          }
        }
      }
      if constexpr (ADJ) {
        if (in) {
          load_x<double, double, WV>(dp + k, xd[v]);
        } else {
#pragma unroll
          for (int e = 0; e < WV; ++e) xd[v][e] = 0.0;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < U; ++v) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        if constexpr (JAC && BF16_MMA) {
          // BF16 weights: each lane's 16 bytes are the B operand of one
          // v_mfma_f32_16x16x32_bf16 (column = lane % 16, K chunk = lane / 16);
          // the FP32 rows go in as BF16 hi + lo parts (x = hi + lo to about
          // 2^-17 relative), two MFMAs per step instead of eight FP32 ones
          const bf16x8 wb = __builtin_bit_cast(bf16x8, wu[v][nb]);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            bf16x8 hi, lo;
#pragma unroll
            for (int e = 0; e < WV; ++e) {
              hi[e] = (bf16)xf[v][rb][e];
              lo[e] = (bf16)(xf[v][rb][e] - (float)hi[e]);
            }
            acc[nb][rb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, wb, acc[nb][rb][0], 0, 0, 0);
            acc[nb][rb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, wb, acc[nb][rb][1], 0, 0, 0);
          }
        } else if constexpr (JAC) {
          A wf[WV];
          Vec16<TW, A>::unpack(wu[v][nb], wf);
#pragma unroll
          for (int e = 0; e < WV; ++e)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[nb][rb][e & 1] = M::mma(xf[v][rb][e], wf[e], acc[nb][rb][e & 1]);
        }
        if constexpr (ADJ) {
          double wd[WV];
          Vec16<TW, double>::unpack(wu[v][nb], wd);
#pragma unroll
          for (int e = 0; e < WV; ++e) adj[nb][e & 1] = fma(wd[e], xd[v][e], adj[nb][e & 1]);
        }
      }
    }
  }
  if constexpr (ADJ) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      double t = adj[nb][0] + adj[nb][1];
      t += __shfl_xor(t, 16, 64);
      t += __shfl_xor(t, 32, 64);
      if (q == 0) red_adj[nb * KSPLIT + wave][c16] = t;
    }
  }
  if constexpr (JAC) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          red[nb * KSPLIT + wave][rb * 16 + M::row(lane, e)][c16] = acc[nb][rb][0][e] + acc[nb][rb][1][e];
  }
  __syncthreads();
  if constexpr (JAC) {
    for (int p = threadIdx.x; p < NB * NR * 16; p += KSPLIT * 64) {
      const int nb = p / (NR * 16);
      const int r = (p >> 4) % NR;
      const int c = p & 15;
      A v = red[nb * KSPLIT][r][c];
#pragma unroll
      for (int w = 1; w < KSPLIT; ++w) v += red[nb * KSPLIT + w][r][c];
      const int j = j0 + nb * 16 + c;
      if (r < a.rows && j < a.N) {
        if (kslices == 1)
          skinny_epilogue<A>(a, a.row0 + r, j, v);
        else
          ((A*)a.part)[((long long)blockIdx.y * a.rows + r) * a.N + j] = v;
      }
    }
  }
  if constexpr (ADJ) {
    if (threadIdx.x < NB * 16) {
      const int nb = threadIdx.x >> 4;
      const int c = threadIdx.x & 15;
      double v = red_adj[nb * KSPLIT][c];
#pragma unroll
      for (int w = 1; w < KSPLIT; ++w) v += red_adj[nb * KSPLIT + w][c];
      const int j = j0 + nb * 16 + c;
      if (j < d.N) {
        if (kslices == 1)
          skinny_epilogue<double>(d, d.row0, j, v);
        else
          ((double*)d.part)[(long long)blockIdx.y * d.N + j] = v;
      }
    }
  }
}

// FP32 Jacobian rows (one to four 16-row blocks, optionally with the FP64
// adjoint row) against packed W^T, rows staged in LDS.  skinny_mfma_kernel
// re-reads the rows from L2 once per weight block: RB x 16 rows of FP32 per
// 16 weight rows, several bytes through L2 per weight byte.  Here a
// workgroup of 8 waves covers 8 weight blocks (128 weight rows) over one K
// slice (blockIdx.y): each chunk of CH K steps of the rows (and of the
// adjoint row) is staged in LDS once and every wave reads it there for its
// own block, so L2 delivers the rows once per workgroup.  A wave owns its
// block over the whole slice (no reduction across waves).
//
// Pipeline, one barrier per chunk: while the MFMAs of chunk c read LDS
// buffer c & 1 and the weights of c from registers, the weights and the rows
// of chunk c + 1 are loaded into registers; the rows then go to the other
// buffer and the barrier publishes them.  The slices' sums go to a.part /
// d.part when there are several, else straight through the epilogue.  Every
// wave runs the same chunk loop, so the barriers are uniform.
//
// LDS layout of a staged row: a pitch of 8 four-byte words beyond the row's
// data, so that the 16 rows a b128 read phase touches start 8 banks apart
// (no conflicts).  FP32 weights: the rows as FP32.  BF16 weights: the rows
// already split into BF16 hi and lo parts (x = hi + lo to about 2^-17
// relative), once per workgroup at staging instead of once per wave, in
// two planes; a lane's 8-element K chunk is one b128 read from each.
template <typename TW, int RB, bool ADJ>
__global__ void __launch_bounds__(512) skinny_rows_lds_kernel(SkinnyArgs a, SkinnyArgs d) {
  constexpr int WV = 16 / (int)sizeof(TW);  // weight elements per 16-byte load
  constexpr int KSTEP = 4 * WV;
  constexpr int NR = 16 * RB;
  constexpr bool BF16_MMA = sizeof(TW) == 2;
  // K steps per staged chunk: 8 (4 for BF16 weights with several row
  // blocks, whose registers would spill at 8)
  constexpr int CH = BF16_MMA && RB >= 2 ? 4 : 8;
  constexpr int CK = CH * KSTEP;
  constexpr int PW = (BF16_MMA ? CK / 2 : CK) + 8;  // row pitch in 4-byte words
  constexpr int PLANE = NR * PW;                    // words per plane (BF16: hi, then lo)
  constexpr int XV = NR * (CK / 4) / 512;           // float4 of staged rows per thread and chunk
  static_assert(XV * 512 == NR * (CK / 4), "rows x chunk must split evenly over 512 threads");
  __shared__ __attribute__((aligned(16))) float xs[2][(BF16_MMA ? 2 : 1) * PLANE];
  __shared__ __attribute__((aligned(16))) double dsh[2][ADJ ? CK : 2];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int c16 = lane & 15;
  const int q = lane >> 4;
  const int nsteps = a.K / KSTEP;
  const int nchunks = (nsteps + CH - 1) / CH;
  const int cper = (nchunks + (int)gridDim.y - 1) / (int)gridDim.y;
  const int c0 = min(nchunks, (int)blockIdx.y * cper);
  const int c1 = min(nchunks, c0 + cper);
  const long long jb = (long long)blockIdx.x * 8 + wave;  // this wave's weight block
  const bool wok = jb * 16 < a.N;
  const TW* wp = (const TW*)a.Wp + (jb * nsteps * 64 + lane) * WV;
  const float* X = (const float*)a.X;
  const double* Z = ADJ ? (const double*)d.X : nullptr;
  floatx4 acc[RB][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb][0] = acc[rb][1] = floatx4{0, 0, 0, 0};
  double adj[2] = {0.0, 0.0};
  uint4 wa[CH], wb[CH];
  float4 xr[XV];
  double zr = 0.0;
  auto load_w = [&](int ch, uint4* w) {
#pragma unroll
    for (int st = 0; st < CH; ++st) {
      const int sg = ch * CH + st;
      w[st] = wok && sg < nsteps ? *(const uint4*)(wp + (long long)sg * 64 * WV) : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto load_rows = [&](int ch) {
    const int k0 = ch * CK;
#pragma unroll
    for (int i = 0; i < XV; ++i) {
      const int t = tid + i * 512;
      const int r = t / (CK / 4);
      const int f = t - r * (CK / 4);  // float4 index within the row's chunk
      xr[i] = r < a.rows && k0 + 4 * f < a.K ? *(const float4*)(X + (long long)r * a.ldx + k0 + 4 * f)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if constexpr (ADJ) zr = tid < CK && k0 + tid < a.K ? Z[k0 + tid] : 0.0;
  };
  auto store_rows = [&](int buf) {
#pragma unroll
    for (int i = 0; i < XV; ++i) {
      const int t = tid + i * 512;
      const int r = t / (CK / 4);
      const int f = t - r * (CK / 4);
      if constexpr (BF16_MMA) {
        const float v[4] = {xr[i].x, xr[i].y, xr[i].z, xr[i].w};
        bf16x4 hi, lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          hi[e] = (bf16)v[e];
          lo[e] = (bf16)(v[e] - (float)hi[e]);
        }
        *(bf16x4*)&xs[buf][r * PW + 2 * f] = hi;
        *(bf16x4*)&xs[buf][PLANE + r * PW + 2 * f] = lo;
      } else {
        *(float4*)&xs[buf][r * PW + 4 * f] = xr[i];
      }
    }
    if constexpr (ADJ) {
      if (tid < CK) dsh[buf][tid] = zr;
    }
  };
  if (c0 < c1) {
    load_w(c0, wa);
    load_rows(c0);
    store_rows(0);
  }
  __syncthreads();
  for (int ch = c0; ch < c1; ++ch) {
    const int buf = (ch - c0) & 1;
    const bool more = ch + 1 < c1;
    if (more) {
      load_w(ch + 1, wb);
      load_rows(ch + 1);
    }
    const float* xb = xs[buf];
#pragma unroll
    for (int st = 0; st < CH; ++st) {
      if constexpr (BF16_MMA) {
        // B operand: this lane's 8 BF16 weights (column c16, K chunk q);
        // A operand: the staged hi and lo parts of the same 8 row elements
        const bf16x8 wv = __builtin_bit_cast(bf16x8, wa[st]);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const float* xp = xb + (rb * 16 + c16) * PW + st * (KSTEP / 2) + 4 * q;
          const bf16x8 hi = *(const bf16x8*)xp;
          const bf16x8 lo = *(const bf16x8*)(xp + PLANE);
          acc[rb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(hi, wv, acc[rb][0], 0, 0, 0);
          acc[rb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lo, wv, acc[rb][1], 0, 0, 0);
        }
      } else {
        float wf[WV];
        Vec16<TW, float>::unpack(wa[st], wf);
        float xe[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const float4 xv = *(const float4*)(xb + (rb * 16 + c16) * PW + st * KSTEP + 4 * q);
          xe[rb][0] = xv.x;
          xe[rb][1] = xv.y;
          xe[rb][2] = xv.z;
          xe[rb][3] = xv.w;
        }
#pragma unroll
        for (int e = 0; e < WV; ++e)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb][e & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(xe[rb][e], wf[e], acc[rb][e & 1], 0, 0, 0);
      }
      if constexpr (ADJ) {
        double wd[WV];
        Vec16<TW, double>::unpack(wa[st], wd);
        const double* zp = &dsh[buf][st * KSTEP + q * WV];
#pragma unroll
        for (int e = 0; e < WV; ++e) adj[e & 1] = fma(wd[e], zp[e], adj[e & 1]);
      }
    }
    if (more) store_rows(buf ^ 1);  // that buffer was last read before the previous barrier
    __syncthreads();
#pragma unroll
    for (int st = 0; st < CH; ++st) wa[st] = wb[st];
  }
  const bool split = gridDim.y > 1;
  const int j = (int)(jb * 16) + c16;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rb * 16 + q * 4 + e;  // accumulator row of element e: 4 (lane / 16) + e
      const float v = acc[rb][0][e] + acc[rb][1][e];
      if (r < a.rows && j < a.N) {
        if (split)
          ((float*)a.part)[((long long)blockIdx.y * a.rows + r) * a.N + j] = v;
        else
          skinny_epilogue<float>(a, a.row0 + r, j, v);
      }
    }
  if constexpr (ADJ) {
    double t = adj[0] + adj[1];
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    if (q == 0 && j < d.N) {
      if (split)
        ((double*)d.part)[(long long)blockIdx.y * d.N + j] = t;
      else
        skinny_epilogue<double>(d, d.row0, j, t);
    }
  }
}

// Sum of the K slices of an MFMA weight stream, in slice order, through the
// epilogue: the a.rows x a.N Jacobian-row block first, then (adj) the
// adjoint row's d.N entries.
template <typename A>
__global__ void skinny_slice_reduce_kernel(SkinnyArgs a, SkinnyArgs d, int kslices, int jac_rows, int adj) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nj = (long long)jac_rows * a.N;
  if (t < nj) {
    const A* P = (const A*)a.part;
    A v = P[t];
    for (int sl = 1; sl < kslices; ++sl) v += P[(long long)sl * nj + t];
    skinny_epilogue<A>(a, a.row0 + (int)(t / a.N), (int)(t % a.N), v);
  } else if (adj && t < nj + d.N) {
    const int j = (int)(t - nj);
    const double* P = (const double*)d.part;
    double v = P[j];
    for (int sl = 1; sl < kslices; ++sl) v += P[(long long)sl * d.N + j];
    skinny_epilogue<double>(d, d.row0, j, v);
  }
}

// Row blocks for `rows` rows (at most kStreamRows).
constexpr int kStreamRows = 64;

// Launch rules for the 5..64-row streams.  Packed FP32 Jacobian rows go to
// skinny_rows_lds_kernel (rows staged in LDS), except one row block on a
// narrow layer.  The remaining packed streams at one row block (the adjoint
// alone, or narrow layers) use two 16-row blocks per wave (each X and
// adjoint fragment read serves both), 16 waves per workgroup for BF16
// weights and 8 otherwise; measured on the 137M network's reverse streams
// against one block per wave: W3^T FP32 69 -> 52 us, BF16 52 -> 41 us.
template <typename TW, typename TX, typename A, int RB, bool JAC, bool ADJ, bool PACKED>
static hipError_t skinny_mfma_launch_p(SkinnyArgs c, SkinnyArgs d, hipStream_t s) {
  const int blocks = (c.N + 15) / 16;
  if constexpr (PACKED && JAC && sizeof(A) == 4 && std::is_same<TX, float>::value) {
   const int groups = (blocks + 7) / 8;
   if (RB >= 2 || groups >= 16) {
    // FP32 Jacobian rows: rows staged in LDS per workgroup of 8 weight
    // blocks (skinny_rows_lds_kernel), K sliced so that the launch is about
    // one workgroup per CU (256; more measured slower, as did a last partial
    // round), every slice keeping 2 chunks or more, within the caller's
    // workspace.  One row block with fewer than 16 workgroups' worth of
    // weight blocks stays on skinny_mfma_kernel (measured faster).
    constexpr int CK = sizeof(TW) == 2 && RB == 1 ? 256 : 128;  // K per chunk
    const int nchunks = (c.K + CK - 1) / CK;
    int ksw = std::max(1, std::min(256 / groups, nchunks / 2));
    while (ksw > 1 && ((long long)ksw * c.rows * c.N > c.part_elems || (ADJ && (long long)ksw * d.N > d.part_elems)))
      --ksw;
    if (!c.part || (ADJ && !d.part)) ksw = 1;
    const int cper = std::max(1, (nchunks + ksw - 1) / ksw);
    ksw = std::max(1, (nchunks + cper - 1) / cper);
    hipLaunchKernelGGL((skinny_rows_lds_kernel<TW, RB, ADJ>), dim3(groups, ksw), dim3(512), 0, s, c, d);
    if (ksw > 1) {
      const long long work = (long long)c.rows * c.N + (ADJ ? d.N : 0);
      hipLaunchKernelGGL(skinny_slice_reduce_kernel<A>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, c, d,
                         ksw, c.rows, (int)ADJ);
    }
    return hipGetLastError();
   }
  }
  if constexpr (PACKED && sizeof(A) == 4 && RB == 1) {
    // One row block and fewer than 512 weight blocks: two blocks per wave
    // (each Jacobian-row and adjoint fragment read serves both) and the K
    // steps split over ksw workgroups as well, up to 2048 waves, every wave
    // keeping 2 steps or more; the slices' sums go to the caller's
    // workspace and are added in slice order by skinny_slice_reduce_kernel.
    constexpr int WV = 16 / (int)sizeof(TW);
    const int nsteps = c.K / (4 * WV);
    const int groups = (blocks + 1) / 2;
    const int jrows = JAC ? c.rows : 0;
    int ksw = (2048 + groups * 8 - 1) / (groups * 8);
    ksw = std::min(ksw, 8);
    while (ksw > 1 && nsteps / ksw < 16) --ksw;
    while (ksw > 1 && ((long long)ksw * jrows * c.N > c.part_elems || (ADJ && (long long)ksw * d.N > d.part_elems)))
      --ksw;
    if (blocks < 512 && ksw >= 2 && (!JAC || c.part) && (!ADJ || d.part)) {
      hipLaunchKernelGGL((skinny_mfma_kernel<TW, TX, A, 8, RB, JAC, ADJ, PACKED, 2>), dim3(groups, ksw), dim3(512), 0,
                         s, c, d);
      const long long work = (long long)jrows * c.N + (ADJ ? d.N : 0);
      hipLaunchKernelGGL(skinny_slice_reduce_kernel<A>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, c, d,
                         ksw, jrows, (int)ADJ);
      return hipGetLastError();
    }
  }
  if constexpr (PACKED && RB == 1) {
    if (blocks >= 512) {
      if constexpr (sizeof(TW) == 2)
        hipLaunchKernelGGL((skinny_mfma_kernel<TW, TX, A, 16, RB, JAC, ADJ, PACKED, 2>), dim3((blocks + 1) / 2),
                           dim3(1024), 0, s, c, d);
      else
        hipLaunchKernelGGL((skinny_mfma_kernel<TW, TX, A, 8, RB, JAC, ADJ, PACKED, 2>), dim3((blocks + 1) / 2),
                           dim3(512), 0, s, c, d);
      return hipGetLastError();
    }
  }
  if (blocks >= 256)
    hipLaunchKernelGGL((skinny_mfma_kernel<TW, TX, A, 8, RB, JAC, ADJ, PACKED>), dim3(blocks), dim3(512), 0, s, c,
                       d);
  else
    hipLaunchKernelGGL((skinny_mfma_kernel<TW, TX, A, 16, RB, JAC, ADJ, PACKED>), dim3(blocks), dim3(1024), 0, s,
                       c, d);
  return hipGetLastError();
}

// The packed weight copy when the caller has one (a.Wp), else the row-major
// weights.
template <typename TW, typename TX, typename A, int RB, bool JAC, bool ADJ>
static hipError_t skinny_mfma_launch_rb(SkinnyArgs c, SkinnyArgs d, hipStream_t s) {
  if (c.Wp) return skinny_mfma_launch_p<TW, TX, A, RB, JAC, ADJ, true>(c, d, s);
  return skinny_mfma_launch_p<TW, TX, A, RB, JAC, ADJ, false>(c, d, s);
}

template <typename TW, typename TX, typename A, bool JAC = true, bool ADJ = false>
static hipError_t skinny_mfma_launch(SkinnyArgs c, SkinnyArgs d, hipStream_t s) {
  if (!JAC) return skinny_mfma_launch_rb<TW, TX, A, 1, JAC, ADJ>(c, d, s);
  switch ((c.rows + 15) / 16) {
    case 1: return skinny_mfma_launch_rb<TW, TX, A, 1, JAC, ADJ>(c, d, s);
    case 2: return skinny_mfma_launch_rb<TW, TX, A, 2, JAC, ADJ>(c, d, s);
    case 3: return skinny_mfma_launch_rb<TW, TX, A, 3, JAC, ADJ>(c, d, s);
    case 4: return skinny_mfma_launch_rb<TW, TX, A, 4, JAC, ADJ>(c, d, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename TW, typename TX, typename A, int R, int JR, int KS>
static hipError_t skinny_ksplit_launch(SkinnyArgs a, hipStream_t s) {
  hipLaunchKernelGGL((skinny_ksplit_kernel<TW, TX, A, R, JR, KS>), dim3((a.N + JR - 1) / JR), dim3(KS * 64), 0,
                     s, a);
  return hipGetLastError();
}

// K split: double it (up to 8 waves) while the launch has fewer than 16384
// waves and every wave still gets at least one vector per lane; two weight
// rows per workgroup (one per workgroup for the output layer).  Measured on
// the 137M network against 4 rows / 8192 waves: forward pass 7-9 % faster.
template <typename TW, typename TX, typename A, int R, int JR>
static hipError_t skinny_launch_jr(SkinnyArgs a, hipStream_t s) {
  constexpr int WV = 16 / (int)sizeof(TW);
  const long long groups = (a.N + JR - 1) / JR;
  const int nvec = a.K / WV;
  int ks = 2;
  while (ks < 8 && groups * ks < 16384 && nvec / (2 * ks) >= 64) ks *= 2;
  switch (ks) {
    case 2: return skinny_ksplit_launch<TW, TX, A, R, JR, 2>(a, s);
    case 4: return skinny_ksplit_launch<TW, TX, A, R, JR, 4>(a, s);
    default: return skinny_ksplit_launch<TW, TX, A, R, JR, 8>(a, s);
  }
}

template <typename TW, typename TX, typename A, int R>
static hipError_t skinny_launch_r(SkinnyArgs a, hipStream_t s) {
  if (a.N < 256) return skinny_launch_jr<TW, TX, A, R, 1>(a, s);
  return skinny_launch_jr<TW, TX, A, R, 2>(a, s);
}

template <typename TW, typename TX, typename A>
static hipError_t skinny_launch(SkinnyArgs a, hipStream_t s) {
  const int total = a.rows;
  const int base = a.row0;
  const char* X = (const char*)a.X;
  for (int done = 0; done < total;) {
    const int left = total - done;
    SkinnyArgs c = a;
    c.row0 = base + done;
    c.X = X + (long long)done * a.ldx * (long long)sizeof(TX);
    hipError_t e;
    int take;
    if (left > 4) {  // 5..64 rows: MFMA stream (one weight read for all rows)
      take = left >= kStreamRows ? kStreamRows : left;
      c.rows = take;
      e = skinny_mfma_launch<TW, TX, A>(c, c, s);
    } else if (left > 2) {
      take = left;
      c.rows = take;
      e = skinny_launch_r<TW, TX, A, 4>(c, s);
    } else if (left == 2) {
      take = 2;
      c.rows = take;
      e = skinny_launch_r<TW, TX, A, 2>(c, s);
    } else {
      take = 1;
      c.rows = 1;
      e = skinny_launch_r<TW, TX, A, 1>(c, s);
    }
    if (e != hipSuccess) return e;
    done += take;
  }
  return hipSuccess;
}

hipError_t launch_skinny(DType wt, DType xt, DType at, SkinnyArgs a, hipStream_t s) {
  if (a.N <= 0 || a.rows <= 0) return hipSuccess;
  if (at == DT_F32) {
    if (xt != DT_F32) return hipErrorInvalidValue;
    if (wt == DT_F32) return skinny_launch<float, float, float>(a, s);
    if (wt == DT_BF16) return skinny_launch<bf16, float, float>(a, s);
    return hipErrorInvalidValue;
  }
  if (xt == DT_F64) {
    if (wt == DT_F32) return skinny_launch<float, double, double>(a, s);
    if (wt == DT_BF16) return skinny_launch<bf16, double, double>(a, s);
    if (wt == DT_F64) return skinny_launch<double, double, double>(a, s);
  } else if (xt == DT_F32) {
    if (wt == DT_F64) return skinny_launch<double, float, double>(a, s);
  }
  return hipErrorInvalidValue;
}

// One point's reverse weight stream for a hidden layer: Jacobian rows `jac`
// (FP32 rows, 0..16 of them; jac.rows = 0 streams the adjoint alone) and the
// FP64 adjoint row `adj` (rows = 1), both against the same W^T.
hipError_t launch_reverse_stream(DType wt, SkinnyArgs jac, SkinnyArgs adj, hipStream_t s) {
  if (adj.rows != 1 || jac.rows < 0 || jac.rows > kStreamRows || adj.N != jac.N || adj.K != jac.K)
    return hipErrorInvalidValue;
  if (adj.N <= 0) return hipSuccess;
  if (jac.rows > 0) {
    if (wt == DT_F32) return skinny_mfma_launch<float, float, float, true, true>(jac, adj, s);
    if (wt == DT_BF16) return skinny_mfma_launch<bf16, float, float, true, true>(jac, adj, s);
  } else {
    if (wt == DT_F32) return skinny_mfma_launch<float, float, float, false, true>(jac, adj, s);
    if (wt == DT_BF16) return skinny_mfma_launch<bf16, float, float, false, true>(jac, adj, s);
  }
  return hipErrorInvalidValue;
}

// Fragment-packed copy of W [N][ldw] (K columns used) for the MFMA weight
// stream: chunk t = (jb * nsteps + st) * 64 + lane holds the 16 bytes that
// lane (c = lane % 16, q = lane / 16) of the stream reads at K step st of
// 16-row block jb: W[16 jb + c][st * 4 V + q V .. + V), V elements of 16
// bytes; rows past N are zero.  One thread per chunk, consecutive threads
// write consecutive chunks.
template <typename T>
__global__ void pack_fragments_kernel(const T* __restrict__ W, long long ldw, int N, int nsteps, long long total,
                                      uint4* __restrict__ Wp) {
  constexpr int V = 16 / (int)sizeof(T);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int lane = (int)(t & 63);
  const long long bs = t >> 6;
  const int st = (int)(bs % nsteps);
  const long long jb = bs / nsteps;
  const long long row = jb * 16 + (lane & 15);
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (row < N) v = *(const uint4*)(W + row * ldw + (long long)st * 4 * V + (lane >> 4) * V);
  Wp[t] = v;
}

hipError_t launch_pack_fragments(DType t, const void* W, long long ldw, int N, int K, void* Wp, hipStream_t s) {
  const int esz = t == DT_F64 ? 8 : t == DT_F32 ? 4 : 2;
  const int V = 16 / esz;
  if (N <= 0 || K <= 0 || K % (4 * V) != 0) return hipErrorInvalidValue;
  const int nsteps = K / (4 * V);
  const long long total = (long long)((N + 15) / 16) * nsteps * 64;
  const long long blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(pack_fragments_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)W, ldw, N,
                         nsteps, total, (uint4*)Wp);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(pack_fragments_kernel<bf16>, dim3((unsigned)blocks), dim3(256), 0, s, (const bf16*)W, ldw, N,
                         nsteps, total, (uint4*)Wp);
      break;
    default:
      hipLaunchKernelGGL(pack_fragments_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)W, ldw,
                         N, nsteps, total, (uint4*)Wp);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- elementwise
template <typename AT>
__global__ void cast_input_kernel(const double* x, int B, int n, AT* xin, int np) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)B * np) return;
  const int b = (int)(i / np);
  const int j = (int)(i % np);
  xin[i] = j < n ? (AT)x[(long long)b * n + j] : (AT)0;
}

hipError_t launch_cast_input(DType at, const double* x, int B, int n, void* xin, int np,
                             hipStream_t s) {
  const long long tot = (long long)B * np;
  if (tot == 0) return hipSuccess;
  const int blocks = (int)((tot + 255) / 256);
  if (at == DT_F64)
    hipLaunchKernelGGL(cast_input_kernel<double>, dim3(blocks), dim3(256), 0, s, x, B, n,
                       (double*)xin, np);
  else
    hipLaunchKernelGGL(cast_input_kernel<float>, dim3(blocks), dim3(256), 0, s, x, B, n,
                       (float*)xin, np);
  return hipGetLastError();
}

// dst = W (rowsp x colsp, zero padded) or W^T (colsp x rowsp), converted to T.
template <typename T>
__global__ void convert_weights_kernel(const double* W, int rows, int cols, T* dst, int rowsp,
                                       int colsp, int transpose) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32;  // column block of W
  const int by = blockIdx.y * 32;  // row block of W
  const int tx = threadIdx.x;
  const int ty = threadIdx.y;
  for (int yy = ty; yy < 32; yy += 8) {
    const int r = by + yy;
    const int c = bx + tx;
    tile[yy][tx] = (r < rows && c < cols) ? W[(long long)r * cols + c] : 0.0;
  }
  __syncthreads();
  if (!transpose) {
    for (int yy = ty; yy < 32; yy += 8) {
      const int r = by + yy;
      const int c = bx + tx;
      if (r < rowsp && c < colsp) dst[(long long)r * colsp + c] = from_d<T>(tile[yy][tx]);
    }
  } else {
    for (int yy = ty; yy < 32; yy += 8) {
      const int c = bx + yy;  // row of W^T
      const int r = by + tx;  // column of W^T
      if (c < colsp && r < rowsp) dst[(long long)c * rowsp + r] = from_d<T>(tile[tx][yy]);
    }
  }
}

hipError_t launch_convert_weights(DType t, const double* W, int rows, int cols, void* dst,
                                  int rowsp, int colsp, bool transpose, hipStream_t s) {
  dim3 grid((colsp + 31) / 32, (rowsp + 31) / 32);
  dim3 block(32, 8);
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(convert_weights_kernel<float>, grid, block, 0, s, W, rows, cols,
                         (float*)dst, rowsp, colsp, (int)transpose);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(convert_weights_kernel<bf16>, grid, block, 0, s, W, rows, cols,
                         (bf16*)dst, rowsp, colsp, (int)transpose);
      break;
    case DT_F64:
      hipLaunchKernelGGL(convert_weights_kernel<double>, grid, block, 0, s, W, rows, cols,
                         (double*)dst, rowsp, colsp, (int)transpose);
      break;
  }
  return hipGetLastError();
}

// out[b*n + j][k] = W1T[j][k] * vec[b][k]: the first tangent P_1 = D_1 W_1
// (or G_1 = diag(s_1) W_1 when layer 1 is the last tangent layer).
template <typename T, typename VT>
__global__ void seed_tangent_kernel(const T* W1T, int n, int dp1, const VT* vec, int B, T* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)B * n * dp1;
  if (i >= tot) return;
  const int k = (int)(i % dp1);
  const long long rj = i / dp1;
  const int j = (int)(rj % n);
  const int b = (int)(rj / n);
  const double w = to_d(W1T[(long long)j * dp1 + k]);
  const double v = (double)vec[(long long)b * dp1 + k];
  out[i] = from_d<T>(w * v);
}

hipError_t launch_seed_tangent(DType t, const void* W1T, int n, int dp1, const void* vec,
                               bool vec_is_double, int B, void* out, hipStream_t s) {
  const long long tot = (long long)B * n * dp1;
  if (tot == 0) return hipSuccess;
  const int blocks = (int)((tot + 255) / 256);
#define NNC_SEED(T, VT)                                                                     \
  hipLaunchKernelGGL((seed_tangent_kernel<T, VT>), dim3(blocks), dim3(256), 0, s, (const T*)W1T, \
                     n, dp1, (const VT*)vec, B, (T*)out)
  switch (t) {
    case DT_F32:
      if (vec_is_double) NNC_SEED(float, double); else NNC_SEED(float, float);
      break;
    case DT_BF16:
      if (vec_is_double) NNC_SEED(bf16, double); else NNC_SEED(bf16, float);
      break;
    case DT_F64:
      NNC_SEED(double, double);
      break;
  }
#undef NNC_SEED
  return hipGetLastError();
}

// Layer-sum seeds of layer 1: T_1 = W_1 (rows of W_1^T per tangent column),
// S_1 = diag(s_1) T_1 and, when a forward product follows, P_1 = D_1 T_1.
// Block row x = tangent row r = b * n + j, y = chunk of 256 16-byte vectors
// along the layer: each thread converts one vector (V elements) of row j of
// W_1^T, elementwise as before, and writes one vector of each output.
template <typename T, typename VT>
__global__ void seed_layersum_kernel(const T* W1T, int n, int dp1, const VT* d1, const double* s1, T* Tc, T* Sc,
                                     long long ldts, T* P) {
  constexpr int V = 16 / (int)sizeof(T);
  const int r = blockIdx.x;
  const int b = r / n;
  const int j = r - b * n;
  const int k0 = (blockIdx.y * blockDim.x + threadIdx.x) * V;
  if (k0 >= dp1) return;  // dp1 is a multiple of 64, so of V
  union Vec {
    uint4 u;
    T e[V];
  };
  Vec w, sv, pv;
  w.u = *(const uint4*)(W1T + (long long)j * dp1 + k0);
  const double* sr = s1 + (long long)b * dp1 + k0;
  const VT* dr = d1 + (long long)b * dp1 + k0;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const double wd = to_d(w.e[e]);
    if (Sc) sv.e[e] = from_d<T>(wd * sr[e]);
    if (P) pv.e[e] = from_d<T>(wd * (double)dr[e]);
  }
  const long long o = (long long)r * ldts + k0;
  *(uint4*)(Tc + o) = w.u;
  if (Sc) *(uint4*)(Sc + o) = sv.u;
  if (P) *(uint4*)(P + (long long)r * dp1 + k0) = pv.u;
}

hipError_t launch_seed_layersum(DType t, const void* W1T, int n, int dp1, const void* d1, const double* s1,
                                int B, void* Tc, void* Sc, long long ldts, void* P, hipStream_t s) {
  const long long rows = (long long)B * n;
  if (rows == 0 || dp1 == 0) return hipSuccess;
  if (rows > 0x7fffffffLL || dp1 % 64 != 0 || ldts % 64 != 0) return hipErrorInvalidValue;
  const int esz = t == DT_F64 ? 8 : t == DT_F32 ? 4 : 2;
  const int vecs = dp1 / (16 / esz);
  const dim3 grid((unsigned)rows, (unsigned)((vecs + 255) / 256));
#define NNC_SEED_LS(T, VT)                                                                              \
  hipLaunchKernelGGL((seed_layersum_kernel<T, VT>), grid, dim3(256), 0, s, (const T*)W1T, n, dp1,          \
                     (const VT*)d1, s1, (T*)Tc, (T*)Sc, ldts, (T*)P)
  switch (t) {
    case DT_F32: NNC_SEED_LS(float, float); break;
    case DT_BF16: NNC_SEED_LS(bf16, float); break;
    case DT_F64: NNC_SEED_LS(double, double); break;
  }
#undef NNC_SEED_LS
  return hipGetLastError();
}

// S_l = diag(s_l) T_l over the layer-sum buffers.  Workgroup (column chunk,
// row group): a chunk is blockDim.x 16-byte vectors of one layer's columns
// (chunks of all layers numbered in turn), a row group kScaleRows rows; each
// thread loads its s_l entries once per point and reuses them down the rows
// (s is FP64, several times the bytes of T).  Each product is rounded as
// where S is formed with T: the first layer's in FP64 (as
// seed_layersum_kernel), the others in the sweep epilogue's type (FP32 for
// FP32 / BF16 buffers, FP64 for FP64) from the stored T.  FP32 and FP64
// thus give the same bits either way; BF16 rounds the later layers' S from
// the stored BF16 T instead of the FP32 accumulator.
constexpr int kScaleRows = 16;

template <typename T, typename V>
__global__ void scale_layersum_kernel(LsScaleArgs a) {
  constexpr int VEC = 16 / (int)sizeof(T);
  const int cw = blockDim.x * VEC;  // columns per chunk
  int cx = blockIdx.x, l = 0;
  for (; l < a.layers; ++l) {
    const int nch = (a.dp[l] + cw - 1) / cw;
    if (cx < nch) break;
    cx -= nch;
  }
  if (l >= a.layers) return;
  const int dp = a.dp[l];
  const int k0 = cx * cw + threadIdx.x * VEC;  // dp is a multiple of VEC: a vector is whole or out
  if (k0 >= dp) return;
  const bool fp64_product = l == 0;  // entry 0 is the network's first layer
  const int r0 = blockIdx.y * kScaleRows;
  const int r1 = min(a.rows, r0 + kScaleRows);
  union Vec {
    uint4 u;
    T e[VEC];
  };
  double sd[VEC];
  int bcur = -1;
#pragma unroll 4
  for (int r = r0; r < r1; ++r) {
    const int b = r / a.n;
    if (b != bcur) {
      const double* sr = a.s[l] + (long long)b * dp + k0;
#pragma unroll
      for (int e = 0; e < VEC; ++e) sd[e] = sr[e];
      bcur = b;
    }
    const long long o = (long long)r * a.ld + a.koff[l] + k0;
    Vec t, q;
    t.u = *(const uint4*)((const T*)a.Tc + o);
    if (fp64_product) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) q.e[e] = from_d<T>(to_d(t.e[e]) * sd[e]);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) q.e[e] = cvt_store<T>((V)to_d(t.e[e]) * (V)sd[e]);
    }
    *(uint4*)((T*)a.Sc + o) = q.u;
  }
}

hipError_t launch_scale_layersum(DType t, const LsScaleArgs& a, hipStream_t s) {
  if (a.rows == 0 || a.layers == 0) return hipSuccess;
  if (a.layers > kMaxScaleLayers || a.rows > 0x7fffffff || a.ld % 64 != 0) return hipErrorInvalidValue;
  const int vec = t == DT_F64 ? 2 : t == DT_F32 ? 4 : 8;
  const int cw = 256 * vec;
  long long chunks = 0;
  for (int l = 0; l < a.layers; ++l) {
    if (a.dp[l] % 64 != 0 || a.koff[l] % 64 != 0) return hipErrorInvalidValue;
    chunks += (a.dp[l] + cw - 1) / cw;
  }
  const dim3 grid((unsigned)chunks, (unsigned)((a.rows + kScaleRows - 1) / kScaleRows));
  switch (t) {
    case DT_F32: hipLaunchKernelGGL((scale_layersum_kernel<float, float>), grid, dim3(256), 0, s, a); break;
    case DT_BF16: hipLaunchKernelGGL((scale_layersum_kernel<bf16, float>), grid, dim3(256), 0, s, a); break;
    case DT_F64: hipLaunchKernelGGL((scale_layersum_kernel<double, double>), grid, dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

__global__ void adj_seed_kernel(const double* lam, const double* zL, int act, int B, int m, int mp,
                                double* zbar, double* sv, const double* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * mp) return;
  const int b = i / mp;
  const int k = i % mp;
  double zb = 0.0, s2 = 0.0;
  if (k < m) {
    const double l = lam[(long long)b * m + k];
    if (act == ACT_SOFTMAX) {
      // g = p * (lambda - p^T lambda): the gradient of lambda^T softmax(z);
      // s holds the diagonal part of its second derivative
      double c = 0.0;
      for (int j = 0; j < m; ++j) c += p[(long long)b * mp + j] * lam[(long long)b * m + j];
      zb = p[i] * (l - c);
      s2 = zb;
    } else {
      const ActVal av = act_eval(act, zL[i]);
      zb = l * av.d1;
      s2 = l * av.d2;
    }
  }
  zbar[i] = zb;
  sv[i] = s2;
}

hipError_t launch_adj_seed(const double* lam, const double* zL, int act, int B, int m, int mp,
                           double* zbar, double* sv, const double* p, hipStream_t s) {
  const int tot = B * mp;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(adj_seed_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, lam, zL, act, B,
                     m, mp, zbar, sv, p);
  return hipGetLastError();
}

// SoftMax of the FP64 output pre-activations, one thread per point: the
// largest entry is subtracted before exponentiating (it cancels).
__global__ void softmax_out_kernel(const double* zL, int B, int m, int mp, const double* y, double* g,
                                   double* p) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double* z = zL + (long long)b * mp;
  double mx = z[0];
  for (int i = 1; i < m; ++i) mx = fmax(mx, z[i]);
  double sum = 0.0;
  for (int i = 0; i < m; ++i) sum += exp(z[i] - mx);
  const double r = 1.0 / sum;
  for (int i = 0; i < mp; ++i) {
    const double pi = i < m ? exp(z[i] - mx) * r : 0.0;
    p[(long long)b * mp + i] = pi;
    if (g && i < m) g[(long long)b * m + i] = y ? y[(long long)b * m + i] - pi : pi;
  }
}

hipError_t launch_softmax_out(const double* zL, int B, int m, int mp, const double* y, double* g, double* p,
                              hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(softmax_out_kernel, dim3((B + 63) / 64), dim3(64), 0, s, zL, B, m, mp, y, g, p);
  return hipGetLastError();
}

// u, v of the SoftMax rank-two term: one thread per tangent row (b, j).
template <typename T>
__global__ void softmax_uv_kernel(const T* Tt, long long ldt, int B, int n, int m, int mp, const double* p,
                                  const double* g, double* u, double* v) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (long long)B * n) return;
  const int b = (int)(r / n);
  double su = 0.0, sv = 0.0;
  for (int i = 0; i < m; ++i) {
    const double t = to_d(Tt[r * ldt + i]);
    su += t * p[(long long)b * mp + i];
    sv += t * g[(long long)b * mp + i];
  }
  u[r] = su;
  v[r] = sv;
}

hipError_t launch_softmax_uv(DType t, const void* Tt, long long ldt, int B, int n, int m, int mp, const double* p,
                             const double* g, double* u, double* v, hipStream_t s) {
  const long long tot = (long long)B * n;
  if (tot == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((tot + 255) / 256);
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(softmax_uv_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)Tt, ldt, B, n, m, mp,
                         p, g, u, v);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(softmax_uv_kernel<bf16>, dim3(blocks), dim3(256), 0, s, (const bf16*)Tt, ldt, B, n, m, mp,
                         p, g, u, v);
      break;
    case DT_F64:
      hipLaunchKernelGGL(softmax_uv_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)Tt, ldt, B, n, m,
                         mp, p, g, u, v);
      break;
  }
  return hipGetLastError();
}

// Jacobian seed rows R[b*m+i][k] = sigma_L'(z_L)[b][i] * W_L[i][k] * sigma_{L-1}'[b][k].
template <typename OT, typename PT>
__global__ void jac_seed_kernel(const double* WL, int m, int kcount, int ldw, const double* d1L,
                                int ldL, const PT* d1prev, int ldp, int B, OT* out, long long ldout,
                                int softmax) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)B * m * ldout;
  if (i >= tot) return;
  const int k = (int)(i % ldout);
  const long long ri = i / ldout;
  const int mi = (int)(ri % m);
  const int b = (int)(ri / m);
  double v = 0.0;
  if (k < kcount) {
    const double* pb = d1L + (long long)b * ldL;
    if (softmax) {
      // row mi of (diag(p) - p p^T) W_L: p_mi (W_L[mi][k] - sum_j p_j W_L[j][k])
      double wbar = 0.0;
      for (int j = 0; j < m; ++j) wbar += pb[j] * WL[(long long)j * ldw + k];
      v = pb[mi] * (WL[(long long)mi * ldw + k] - wbar);
    } else {
      v = pb[mi] * WL[(long long)mi * ldw + k];
    }
    if (d1prev) v *= (double)d1prev[(long long)b * ldp + k];
  }
  out[i] = (OT)v;
}

hipError_t launch_jac_seed(DType at, const double* WL, int m, int K, int Kp, const void* d1L,
                           int ldL, const void* d1prev, int ldp, int B, void* R, bool out_double,
                           bool softmax, hipStream_t s) {
  // out_double: write J (ld = K = n) directly; otherwise R rows of width Kp.
  const long long ldout = out_double ? K : Kp;
  const long long tot = (long long)B * m * ldout;
  if (tot == 0) return hipSuccess;
  const int blocks = (int)((tot + 255) / 256);
  if (out_double) {
    hipLaunchKernelGGL((jac_seed_kernel<double, double>), dim3(blocks), dim3(256), 0, s, WL, m, K,
                       Kp, (const double*)d1L, ldL, (const double*)nullptr, ldp, B, (double*)R,
                       ldout, (int)softmax);
  } else if (at == DT_F64) {
    hipLaunchKernelGGL((jac_seed_kernel<double, double>), dim3(blocks), dim3(256), 0, s, WL, m, K,
                       Kp, (const double*)d1L, ldL, (const double*)d1prev, ldp, B, (double*)R,
                       ldout, (int)softmax);
  } else {
    hipLaunchKernelGGL((jac_seed_kernel<float, float>), dim3(blocks), dim3(256), 0, s, WL, m, K,
                       Kp, (const double*)d1L, ldL, (const float*)d1prev, ldp, B, (float*)R, ldout,
                       (int)softmax);
  }
  return hipGetLastError();
}

// H = 0.5 * (P + P^T) summed over split partials, plus obj * diag(q).  With
// symtile > 0 only the partial tiles on or below the block diagonal were
// written: entries below it come from P[r][c], above it from P[c][r], and
// diagonal tiles are symmetrised; the unwritten tiles are never read.
__global__ void finalize_h_kernel(const double* part, int splits, long long sstride, int n,
                                  double obj, const double* q, double* H, int symtile, const double* u,
                                  const double* vv) {
  __shared__ double ta[32][33];
  __shared__ double tb[32][33];
  const int b = blockIdx.z;
  const int I = blockIdx.y * 32;
  const int J = blockIdx.x * 32;
  const int tx = threadIdx.x;
  const long long base = (long long)b * n * n;
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    double sa = 0.0, sb = 0.0;
    const int ra = I + yy, ca = J + tx;
    const int rb = J + yy, cb = I + tx;
    const bool la = ra < n && ca < n && (symtile <= 0 || ra / symtile >= ca / symtile);
    const bool lb = rb < n && cb < n && (symtile <= 0 || rb / symtile >= cb / symtile);
    // up to 8 split partials loaded back to back, then added in split order
    for (int sp0 = 0; sp0 < splits; sp0 += 8) {
      double va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double* P = part + (long long)(sp0 + u) * sstride + base;
        va[u] = la && sp0 + u < splits ? P[(long long)ra * n + ca] : 0.0;
        vb[u] = lb && sp0 + u < splits ? P[(long long)rb * n + cb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (la && sp0 + u < splits) sa += va[u];
        if (lb && sp0 + u < splits) sb += vb[u];
      }
    }
    ta[yy][tx] = sa;
    tb[yy][tx] = sb;
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    const int r = I + yy, c = J + tx;
    if (r < n && c < n) {
      double v;
      if (symtile > 0 && r / symtile != c / symtile)
        v = r / symtile > c / symtile ? ta[yy][tx] : tb[tx][yy];
      else
        v = 0.5 * (ta[yy][tx] + tb[tx][yy]);
      if (r == c && q) v += obj * q[r];
      if (u) {
        // products rounded on their own (contraction into fused multiply-adds
        // off), so that (r, c) and (c, r) round the same two products and H
        // stays exactly symmetric
#pragma clang fp contract(off)
        const long long rb = (long long)b * n;
        const double t1 = u[rb + r] * vv[rb + c];
        const double t2 = vv[rb + r] * u[rb + c];
        v -= r <= c ? t1 + t2 : t2 + t1;
      }
      H[base + (long long)r * n + c] = v;
    }
  }
}

hipError_t launch_finalize_h(const double* part, int splits, long long split_stride, int B, int n,
                             double obj, const double* q, double* H, int symtile, const double* u,
                             const double* v, hipStream_t s) {
  if (B == 0 || n == 0) return hipSuccess;
  dim3 grid((n + 31) / 32, (n + 31) / 32, B);
  hipLaunchKernelGGL(finalize_h_kernel, grid, dim3(32, 8), 0, s, part, splits, split_stride, n,
                     obj, q, H, symtile, u, v);
  return hipGetLastError();
}

// Lower triangle of each n x n matrix, row by row:
// Hp[b][i(i+1)/2 + j] = H[b][i][j] for j <= i.  One thread per packed entry
// (consecutive threads write consecutive entries); the row i of entry p is
// the largest i with i(i+1)/2 <= p, from the square root and corrected in
// integers.
__global__ void pack_lower_kernel(const double* __restrict__ H, int n, long long tri, long long total,
                                  double* __restrict__ Hp) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const long long b = t / tri;
  const long long p = t - b * tri;
  long long i = (long long)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i > 0 && i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const long long j = p - i * (i + 1) / 2;
  Hp[t] = H[(b * n + i) * n + j];
}

hipError_t launch_pack_lower(const double* H, int B, int n, double* Hp, hipStream_t s) {
  const long long tri = (long long)n * (n + 1) / 2;
  const long long total = tri * B;
  if (total == 0) return hipSuccess;
  const long long blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pack_lower_kernel, dim3((unsigned)blocks), dim3(256), 0, s, H, n, tri, total, Hp);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
  if (i < ntail) tail[i] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes % 16;
  const size_t work = n16 > ntail ? n16 : ntail;
  const size_t blocks = (work + 255) / 256;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}

__global__ void check_finite_kernel(const double* p, size_t count, int* flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && !isfinite(p[i])) atomicOr(flag, 1);
}

// Largest |a - ref| and largest |ref| over an M x N matrix (row stride ld),
// as the bit patterns of non-negative floats combined with integer atomicMax
// (order-independent: the result does not depend on scheduling).  out[0],
// out[1] must start at zero.
template <typename T>
__global__ void max_abs_diff_kernel(const T* __restrict__ a, const T* __restrict__ ref, int M, int N, long long ld,
                                    unsigned* out) {
  __shared__ float sd[256], sr[256];
  float d = 0.f, r = 0.f;
  const long long total = (long long)M * N;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long o = (i / N) * ld + i % N;
    const float x = (float)a[o], y = (float)ref[o];
    const float e = fabsf(x - y);
    d = fmaxf(d, e != e ? INFINITY : e);  // a NaN difference counts as infinite
    r = fmaxf(r, fabsf(y));
  }
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sd[threadIdx.x] = fmaxf(sd[threadIdx.x], sd[threadIdx.x + w]);
      sr[threadIdx.x] = fmaxf(sr[threadIdx.x], sr[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, __float_as_uint(sd[0]));
    atomicMax(out + 1, __float_as_uint(sr[0]));
  }
}

hipError_t launch_max_abs_diff(DType t, const void* a, const void* ref, int M, int N, long long ld, unsigned* out,
                               hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const long long total = (long long)M * N;
  const int blocks = (int)std::min<long long>((total + 255) / 256, 1024);
  switch (t) {
    case DT_F32:
      hipLaunchKernelGGL(max_abs_diff_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)a,
                         (const float*)ref, M, N, ld, out);
      break;
    case DT_BF16:
      hipLaunchKernelGGL(max_abs_diff_kernel<bf16>, dim3(blocks), dim3(256), 0, s, (const bf16*)a, (const bf16*)ref,
                         M, N, ld, out);
      break;
    default:
      hipLaunchKernelGGL(max_abs_diff_kernel<double>, dim3(blocks), dim3(256), 0, s, (const double*)a,
                         (const double*)ref, M, N, ld, out);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* p, size_t count, int* flag, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p,
                     count, flag);
  return hipGetLastError();
}

}  // namespace nnc
