#pragma once
// MFMA GEMM kernels for gfx950 (CDNA4) with fused tangent-sweep epilogues.
// Included by one translation unit per element type (gemm_f32.hip,
// gemm_bf16.hip, gemm_f64.hip) so the instantiations compile in parallel;
// gemm.hip holds the tiling registry and the type dispatch.
//
// C[M][N] = A[M][K] * B[N][K]^T; both operands are K-contiguous, so every
// layer of the forward-tangent sweep (B = W_{l+1}) and of the reverse-tangent
// sweep (B = W_l^T, a transposed weight copy) is the same "NT" product.
//
// Structure (per workgroup, WM x WN waves of 64 lanes):
//   * a BM x BN output tile, BM = WM*FM*16, BN = WN*FN*16, each wave owning
//     FM x FN blocks of 16x16 accumulated by v_mfma 16x16 instructions;
//   * K advanced in tiles of 128 bytes per row (32 fp32 / 64 bf16 / 16 fp64),
//     staged global -> registers -> LDS with a double-buffered LDS ring and a
//     single barrier per K tile; the next tile's global loads are issued
//     before the current tile's MFMAs so their latency is hidden;
//   * LDS rows of 128 bytes with the 16-byte chunks XOR-swizzled per row, so
//     both the stores (two rows x 8 chunks per 16 lanes) and the 16-row
//     fragment reads are free of bank conflicts;
//   * each lane reads one 16-byte vector of A and of B per 64-byte k-group
//     and feeds it to 4 (fp32), 1 (bf16 16x16x32) or 2 (fp64) MFMAs: lane
//     group q = lane/16 holds k in [q*16B, (q+1)*16B) of the group, the same
//     k permutation for A and B, so the sum over k is unchanged;
//   * workgroup -> tile mapping is XCD-aware: consecutive workgroup ids land
//     on different XCDs (round-robin dispatch), so ids are remapped to give
//     each XCD a contiguous run of tiles that share weight (B) tiles in its L2.
//
// The tilings from kFirstDmaCfg on stage K tiles by LDS DMA instead
// (gemm_dma.hip, FP32 and BF16); the autotuner picks among all of them.
#include "gemm_common.h"

namespace nnc {

// One BM x BN output tile (tile id t, K split `split`) of the NT product.
// PF = prefetch distance in K tiles: 1 loads tile k+1 while tile k is
// multiplied; 2 keeps two register sets and loads tile k+2, so a load has two
// tiles' worth of MFMA time to arrive (BF16 spends a quarter of FP32's MFMA
// instructions per staged byte, which leaves PF = 1 waiting on memory).
template <typename T, int WM, int WN, int FM, int FN, bool ACC64, int PF = 1, bool SWEEP = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g0, int t, int split, char* smem) {
  static_assert(PF == 1 || PF == 2, "prefetch distance 1 or 2");
  using Ops = MfmaOps<T>;
  using Acc = typename Ops::Acc;
  constexpr int NT = WM * WN * 64;
  constexpr int BM = WM * FM * 16;
  constexpr int BN = WN * FN * 16;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int BK = 8 * VEC;  // 128 bytes of K per row per tile
  constexpr int ROWB = 128;    // LDS row pitch (bytes); 16-byte chunks XOR-swizzled
  constexpr int ROWS = BM + BN;
  constexpr int CHUNKS = ROWS * 8;
  constexpr int CPT = (CHUNKS + NT - 1) / NT;
  constexpr int STAGE = ROWS * ROWB;

  GemmArgs g = g0;
  int tm, tn;
  locate_tile<T>(g, t, tm, tn);
  const int m0 = tm * BM;
  const int n0 = tn * BN;
  const int kbeg = split * g.kper;
  const int kend = min(g.K, kbeg + g.kper);
  const int nk = (kend - kbeg) / BK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  // Global -> LDS staging.  Thread tid moves 16-byte chunk kc = tid % 8 of
  // rows r0 + p * RSTEP (p = 0..CPT-1) of the stacked [A rows; B rows] tile.
  // Loads are raw buffer loads through one buffer resource per operand whose
  // size is the operand's extent (M * lda or N * ldb elements): a row outside
  // the operand gets an offset past that extent and the hardware returns
  // zeros.  No branch surrounds a load, so the compiler counts outstanding
  // loads exactly (with PF = 2 it then waits only for the older register
  // set).  Operands are below 2 GiB (checked when a network is created), so
  // the out-of-range offset 2^31 plus any K offset stays out of range.
  constexpr int RSTEP = NT / 8;
  constexpr unsigned OOB = 0x80000000u;
  const int r0 = tid >> 3;
  const int kc = tid & 7;
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      (void*)g.A, (short)0, (int)((unsigned long long)g.M * g.lda * sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      (void*)g.B, (short)0, (int)((unsigned long long)g.N * g.ldb * sizeof(T)), 0x00020000);
  unsigned voff[CPT];  // byte offset of this thread's chunk of row r0 + p * RSTEP at kt = 0
#pragma unroll
  for (int p = 0; p < CPT; ++p) {
    const int row = r0 + p * RSTEP;
    const unsigned kb = (unsigned)((kbeg + kc * VEC) * (int)sizeof(T));
    if (row < BM) {
      voff[p] = m0 + row < g.M ? (unsigned)((m0 + row) * (unsigned long long)g.lda * sizeof(T)) + kb : OOB;
    } else {
      voff[p] = (row < ROWS && n0 + row - BM < g.N)
                    ? (unsigned)((n0 + row - BM) * (unsigned long long)g.ldb * sizeof(T)) + kb
                    : OOB;
    }
  }
  // Chunk c of stacked-tile row r lives at chunk slot c ^ swz(r), swz(r) =
  // r & 6.  gfx950's LDS has 64 four-byte banks and serves a 16-byte access
  // 16 lanes per cycle, in the lane groups {0-3, 12-15, 20-27},
  // {4-11, 16-19, 28-31} and the same plus 32 (measured with the bank-conflict
  // counter).  With this key each group of a fragment read (16 rows, one
  // chunk each) and of a store (8 rows x 8 chunks per wave) covers the 16
  // distinct 16-byte slots of a 256-byte bank line.  Rows a thread touches
  // differ by multiples of 16, so the key is a per-thread constant.
  const int swz_st = r0 & 6;
  const int lds0 = r0 * ROWB + ((kc ^ swz_st) * 16);

  auto gload = [&](int kt, uint4 (&regs)[CPT]) {
    const unsigned kbytes = (unsigned)(kt * BK * (int)sizeof(T));
#pragma unroll
    for (int p = 0; p < CPT; ++p) {
      // which operand a chunk belongs to is known at compile time except in
      // the one group that straddles BM: there both loads are issued, the
      // one for the other operand out of range (zeros), and OR-ed
      if ((p + 1) * RSTEP <= BM) {  // folds once the loop is unrolled
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rsA, (int)(voff[p] + kbytes), 0, 0);
        regs[p] = make_uint4(w[0], w[1], w[2], w[3]);
      } else if (p * RSTEP >= BM) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rsB, (int)(voff[p] + kbytes), 0, 0);
        regs[p] = make_uint4(w[0], w[1], w[2], w[3]);
      } else {
        const bool is_a = r0 + p * RSTEP < BM;
        const unsigned oa = is_a ? voff[p] + kbytes : OOB;
        const unsigned ob = is_a ? OOB : voff[p] + kbytes;
        const auto wa = __builtin_amdgcn_raw_buffer_load_b128(rsA, (int)oa, 0, 0);
        const auto wb = __builtin_amdgcn_raw_buffer_load_b128(rsB, (int)ob, 0, 0);
        regs[p] = make_uint4(wa[0] | wb[0], wa[1] | wb[1], wa[2] | wb[2], wa[3] | wb[3]);
      }
    }
  };
  auto sstore = [&](int buf, const uint4 (&regs)[CPT]) {
#pragma unroll
    for (int p = 0; p < CPT; ++p) {
      if (r0 + p * RSTEP < ROWS) *(uint4*)(smem + buf * STAGE + lds0 + p * RSTEP * ROWB) = regs[p];
    }
  };

  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};
  double acc64[ACC64 ? FM : 1][ACC64 ? FN : 1][4];
  if constexpr (ACC64) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc64[i][j][e] = 0.0;
  }

  uint4 ra[CPT];
  uint4 rb[PF == 2 ? CPT : 1];
  if (nk > 0) {
    gload(0, ra);
    sstore(0, ra);
  }
  if constexpr (PF == 2) {
    if (nk > 1) gload(1, rb);
  }
  __syncthreads();

  const int arow = wm * FM * 16 + (lane & 15);
  const int brow = BM + wn * FN * 16 + (lane & 15);
  const int swz_ld = lane & 6;  // swz of rows arow + 16i and brow + 16j
  const int kofs0 = (((lane >> 4) + 0) ^ swz_ld) * 16;  // k-group 0: chunks 0..3
  const int kofs1 = (((lane >> 4) + 4) ^ swz_ld) * 16;  // k-group 1: chunks 4..7

  // MFMAs over the K tile in LDS buffer `buf`
  auto compute = [&](int buf) {
    const char* sb = smem + buf * STAGE;
#pragma unroll
    for (int kg = 0; kg < 2; ++kg) {
      uint4 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = *(const uint4*)(sb + (arow + i * 16) * ROWB + (kg ? kofs1 : kofs0));
#pragma unroll
      for (int j = 0; j < FN; ++j) bfr[j] = *(const uint4*)(sb + (brow + j * 16) * ROWB + (kg ? kofs1 : kofs0));
      // step-major order: consecutive MFMAs update different accumulators
#pragma unroll
      for (int st = 0; st < Ops::STEPS; ++st)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) Ops::mma(acc[i][j], af[i], bfr[j], st);
    }
  };
  // ACC64: the FP32 MFMA sums are added into FP64 accumulators after every
  // FOLD K tiles (and after the last): 256 K terms for BF16, 64 for FP32 --
  // FP64 across chunks of K, at a fraction of the conversions and FP64 adds
  // that folding every tile costs (for BF16 as many cycles as the MFMAs).
  // The fold points depend only on the tile index: deterministic.
  constexpr int FOLD = sizeof(T) == 2 ? 4 : 2;
  auto fold = [&](int kt) {
    if constexpr (ACC64) {
      if ((kt + 1) % FOLD == 0 || kt + 1 == nk) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) acc64[i][j][e] += (double)acc[i][j][e];
            acc[i][j] = Acc{0, 0, 0, 0};
          }
      }
    }
  };

  if constexpr (PF == 1) {
    for (int kt = 0; kt < nk; ++kt) {
      if (kt + 1 < nk) gload(kt + 1, ra);
      compute(kt & 1);
      fold(kt);
      if (kt + 1 < nk) sstore((kt + 1) & 1, ra);
      __syncthreads();
    }
  } else {
    // tile k lives in LDS buffer k & 1; the loop is unrolled by two so each
    // register set has a fixed role: ra carries even tiles, rb odd ones.
    for (int kt = 0; kt < nk; kt += 2) {
      if (kt + 2 < nk) gload(kt + 2, ra);
      compute(0);
      fold(kt);
      if (kt + 1 < nk) sstore(1, rb);
      __syncthreads();
      if (kt + 1 >= nk) break;
      if (kt + 3 < nk) gload(kt + 3, rb);
      compute(1);
      fold(kt + 1);
      if (kt + 2 < nk) sstore(0, ra);
      __syncthreads();
    }
  }

  finish_tile<T, WM, WN, FM, FN, ACC64, SWEEP>(g, acc, acc64, m0, n0, wm, wn, lane, split);
}

template <typename T, int WM, int WN, int FM, int FN, bool ACC64, int PF = 1>
__global__ void __launch_bounds__(WM * WN * 64) gemm_nt_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) char smem[TileShape<T, WM, WN, FM, FN>::SMEM];
  const int t = xcd_remap(blockIdx.x, gemm_tiles_per_split(g));
  gemm_tile<T, WM, WN, FM, FN, ACC64, PF>(g, t, blockIdx.y, smem);
}

// Persistent grouped GEMM: one launch walks the tiles of several independent
// products (one per network of a batch, possibly with K splits).  Workgroup w
// takes work items w, w + gridDim.x, ...; item -> (group, split, tile) via the
// prefix offsets.  Groups are ordered by decreasing cost per tile so the
// static round-robin assignment stays balanced.  Only tangent-sweep products
// (and their K-split partials) are grouped, so only their epilogues are built.
template <typename T, int WM, int WN, int FM, int FN, bool ACC64, int PF = 1>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_grouped_kernel(const GemmArgs* __restrict__ groups, const int* __restrict__ offsets, int ngroups) {
  __shared__ __attribute__((aligned(16))) char smem[TileShape<T, WM, WN, FM, FN>::SMEM];
  const int total = offsets[ngroups];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int gi = 0;
    while (gi + 1 < ngroups && offsets[gi + 1] <= w) ++gi;
    const GemmArgs g = groups[gi];
    const int local = w - offsets[gi];
    const int tiles = gemm_tiles_per_split(g);
    const int split = local / tiles;
    const int t = xcd_remap(local % tiles, tiles);
    gemm_tile<T, WM, WN, FM, FN, ACC64, PF, true>(g, t, split, smem);
    __syncthreads();
  }
}

// K-split reduction: the sweep GEMM ran as `splits` K slices writing
// partials part[s][row][col] (row stride N; FP32, or FP64 for FP64 GEMMs);
// add them in slice order and apply the GEMM's own fused epilogue.  One
// thread per output element, consecutive threads on consecutive columns
// (coalesced partial reads and output writes).
template <typename T, int EPI>
__global__ void __launch_bounds__(256) splitk_reduce_kernel(GemmArgs g, const void* __restrict__ partv,
                                                            int splits) {
  using P = typename MfmaOps<T>::AccT;  // float, or double for FP64 GEMMs
  const P* part = (const P*)partv;
  const long long MN = (long long)g.M * g.N;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= MN) return;
  P v = part[i];
  for (int s = 1; s < splits; ++s) v += part[s * MN + i];
  const int row = (int)(i / g.N);
  const int col = (int)(i - (long long)row * g.N);
  gemm_epilogue<T, P, EPI>(g, row, col, v, 0);
}

template <typename T>
static hipError_t splitk_reduce_typed(GemmArgs g, const void* part, int splits, hipStream_t s) {
  const long long MN = (long long)g.M * g.N;
  const long long blocks = (MN + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)blocks);
  switch (g.epi) {
    case EPI_FWD_T: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_FWD_T>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_FWD_G: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_FWD_G>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_REV_G: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_REV_G>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_FWD_LS: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_FWD_LS>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_FWD_LT: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_FWD_LT>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_JAC_R: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_JAC_R>), grid, dim3(256), 0, s, g, part, splits); break;
    case EPI_F64: hipLaunchKernelGGL((splitk_reduce_kernel<T, EPI_F64>), grid, dim3(256), 0, s, g, part, splits); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int WM, int WN, int FM, int FN, bool ACC64, int PF = 1>
static hipError_t launch_cfg(GemmArgs g, int splits, hipStream_t s) {
  constexpr int BM = WM * FM * 16;
  constexpr int BN = WN * FN * 16;
  g.tiles_m = (g.M + BM - 1) / BM;
  g.tiles_n = (g.N + BN - 1) / BN;
  if (g.sym > 0 && (BM != g.sym || BN != g.sym || g.M != g.N)) return hipErrorInvalidValue;
  dim3 grid(gemm_tiles_per_split(g), splits);
  hipLaunchKernelGGL((gemm_nt_kernel<T, WM, WN, FM, FN, ACC64, PF>), grid, dim3(WM * WN * 64), 0, s, g);
  return hipGetLastError();
}

template <typename T, int WM, int WN, int FM, int FN, bool ACC64, int PF = 1>
static hipError_t launch_grouped_cfg(const GemmArgs* groups, const int* offsets, int ngroups, int grid,
                                     hipStream_t s) {
  hipLaunchKernelGGL((gemm_grouped_kernel<T, WM, WN, FM, FN, ACC64, PF>), dim3(grid), dim3(WM * WN * 64), 0,
                     s, groups, offsets, ngroups);
  return hipGetLastError();
}

template <typename T, bool ACC64>
static hipError_t launch_grouped_typed(int cfg, const GemmArgs* groups, const int* offsets, int ngroups,
                                       int grid, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_grouped_cfg<T, 2, 2, 4, 4, ACC64>(groups, offsets, ngroups, grid, s);
    case 1: return launch_grouped_cfg<T, 1, 4, 13, 1, ACC64>(groups, offsets, ngroups, grid, s);
    case 3: return launch_grouped_cfg<T, 2, 2, 2, 2, ACC64>(groups, offsets, ngroups, grid, s);
    case 5: return launch_grouped_cfg<T, 1, 4, 7, 2, ACC64>(groups, offsets, ngroups, grid, s);
    default: break;
  }
  if constexpr (!ACC64) {  // 8-wave tilings: one workgroup per CU
    switch (cfg) {
      case 2: return launch_grouped_cfg<T, 1, 8, 13, 1, false>(groups, offsets, ngroups, grid, s);
      case 4: return launch_grouped_cfg<T, 2, 4, 8, 4, false>(groups, offsets, ngroups, grid, s);
      case 6: return launch_grouped_cfg<T, 2, 4, 4, 4, false>(groups, offsets, ngroups, grid, s);
      case 7: return launch_grouped_cfg<T, 1, 8, 7, 2, false>(groups, offsets, ngroups, grid, s);
      case 9: return launch_grouped_cfg<T, 1, 8, 13, 1, false, 2>(groups, offsets, ngroups, grid, s);
      case 11: return launch_grouped_cfg<T, 1, 8, 7, 2, false, 2>(groups, offsets, ngroups, grid, s);
      case 13: return launch_grouped_cfg<T, 2, 4, 4, 4, false, 2>(groups, offsets, ngroups, grid, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

template <typename T, bool ACC64>
static hipError_t launch_typed(int cfg, GemmArgs g, int splits, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_cfg<T, 2, 2, 4, 4, ACC64>(g, splits, s);
    case 1: return launch_cfg<T, 1, 4, 13, 1, ACC64>(g, splits, s);
    case 2: return launch_cfg<T, 1, 8, 13, 1, ACC64>(g, splits, s);
    case 3: return launch_cfg<T, 2, 2, 2, 2, ACC64>(g, splits, s);
    case 4: return launch_cfg<T, 2, 4, 8, 4, ACC64>(g, splits, s);
    case 5: return launch_cfg<T, 1, 4, 7, 2, ACC64>(g, splits, s);
    case 6: return launch_cfg<T, 2, 4, 4, 4, ACC64>(g, splits, s);
    case 7: return launch_cfg<T, 1, 8, 7, 2, ACC64>(g, splits, s);
    default: break;
  }
  if constexpr (!ACC64) {  // tilings without FP64 cross-tile accumulation
    switch (cfg) {
      case 8: return launch_cfg<T, 2, 2, 4, 4, false, 2>(g, splits, s);
      case 9: return launch_cfg<T, 1, 8, 13, 1, false, 2>(g, splits, s);
      case 10: return launch_cfg<T, 1, 4, 7, 2, false, 2>(g, splits, s);
      case 11: return launch_cfg<T, 1, 8, 7, 2, false, 2>(g, splits, s);
      case 12: return launch_cfg<T, 2, 4, 8, 4, false, 2>(g, splits, s);
      case 13: return launch_cfg<T, 2, 4, 4, 4, false, 2>(g, splits, s);
      case 14: return launch_cfg<T, 1, 4, 7, 4, false, 1>(g, splits, s);
      case 15: return launch_cfg<T, 2, 2, 4, 8, false, 1>(g, splits, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// Configurations the autotuner tries (the larger tiles that spill

// Entry points of one element type, defined by the per-type translation units.
#define NNC_GEMM_TYPED_ENTRY_POINTS(T, SUF)                                                               \
  hipError_t gemm_launch_##SUF(int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s) {              \
    if constexpr (sizeof(T) == 8) {                                                                       \
      if (acc64) return hipErrorInvalidValue; /* FP64 MFMA already accumulates in FP64 */                 \
      return launch_typed<T, false>(cfg, g, splits, s);                                                   \
    } else {                                                                                              \
      return acc64 ? launch_typed<T, true>(cfg, g, splits, s) : launch_typed<T, false>(cfg, g, splits, s); \
    }                                                                                                     \
  }                                                                                                       \
  hipError_t gemm_grouped_##SUF(int cfg, bool acc64, const GemmArgs* groups, const int* offsets,          \
                                int ngroups, int grid, hipStream_t s) {                                   \
    if constexpr (sizeof(T) == 8) {                                                                       \
      if (acc64) return hipErrorInvalidValue;                                                             \
      return launch_grouped_typed<T, false>(cfg, groups, offsets, ngroups, grid, s);                      \
    } else {                                                                                              \
      return acc64 ? launch_grouped_typed<T, true>(cfg, groups, offsets, ngroups, grid, s)                \
                   : launch_grouped_typed<T, false>(cfg, groups, offsets, ngroups, grid, s);              \
    }                                                                                                     \
  }                                                                                                       \
  hipError_t gemm_splitk_##SUF(GemmArgs g, const void* part, int splits, hipStream_t s) {                 \
    return splitk_reduce_typed<T>(g, part, splits, s);                                                    \
  }

}  // namespace nnc
