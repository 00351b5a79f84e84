// MFMA GEMM tiles staged by LDS DMA (gfx950 buffer_load_dwordx4 ... lds).
//
// Same product, tile shapes, MFMA issue order, LDS row layout and epilogues
// as the register-staged kernel in gemm.hip; only the global -> LDS staging
// differs.  Each wave's buffer loads write their 16-byte chunks straight into
// LDS, so staging takes no VGPRs and no ds_write instructions, and NS LDS
// stages (2 to 4) keep NS - 1 K tiles in flight while one is multiplied.
//
//   * A wave's DMA load writes its 64 lanes' chunks to 1024 consecutive LDS
//     bytes (lane l at byte 16 l: 8 rows of 128 bytes), so the XOR swizzle
//     of the register-staged kernel moves to the global side: the lane that
//     fills slot c of row r loads global chunk c ^ swz(r).  Fragment reads
//     are unchanged.
//   * The stages are separate LDS arrays.  The compiler then waits, before a
//     fragment read, only for the DMA loads into that stage; the explicit
//     wait before each barrier covers this wave's loads of the tile about to
//     be read (the barrier then makes every wave's chunks visible) and leaves
//     the newer tiles in flight.  The barrier carries no memory fence, since
//     a fence would wait for all outstanding loads.
//   * Rows outside an operand read as zeros through the buffer resource's
//     range check (offset 2^31, as in gemm.hip), so no branch surrounds a
//     load and every wave issues the same number of loads per tile.
#include "gemm_common.h"

namespace nnc {

typedef __attribute__((address_space(3))) void* lds_ptr;

// s_waitcnt immediate that waits until at most n vector-memory operations of
// this wave are outstanding (expcnt and lgkmcnt left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// Workgroup barrier without a memory fence (the compiler barriers keep LDS
// accesses on their side of it).
__device__ __forceinline__ void barrier_nofence() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// LDS bytes of one stage of a tiling
template <typename T, int WM, int WN, int FM, int FN>
constexpr int dma_stage_bytes() { return (WM * FM * 16 + WN * FN * 16) * 128; }

// One BM x BN output tile (tile id t, K split `split`) staged through the
// LDS arrays st0..st3 (distinct arrays of the calling kernel).  SWEEP builds
// only the tangent-sweep epilogues (grouped launches).
template <typename T, int WM, int WN, int FM, int FN, int NS, int U, bool SWEEP>
__device__ __forceinline__ void dma_tile(const GemmArgs& g0, int t, int split, char* st0, char* st1, char* st2,
                                         char* st3) {
  static_assert(NS >= 2 && NS <= 4, "2 to 4 LDS stages");
  static_assert(U % NS == 0, "the loop body holds whole rounds of stages");
  using Ops = MfmaOps<T>;
  using Acc = typename Ops::Acc;
  constexpr int NT = WM * WN * 64;
  constexpr int BM = WM * FM * 16;
  constexpr int BN = WN * FN * 16;
  constexpr int VEC = 16 / (int)sizeof(T);
  constexpr int BK = 8 * VEC;  // 128 bytes of K per row per tile
  constexpr int ROWB = 128;
  constexpr int ROWS = BM + BN;
  constexpr int RSTEP = NT / 8;  // stacked-tile rows per load group (8 per wave)
  constexpr int CPT = ROWS / RSTEP;  // DMA loads per wave per K tile
  static_assert(ROWS % RSTEP == 0 && BM % RSTEP == 0, "load groups must not straddle operands");
  static_assert(CPT * (NS - 2) < 64, "outstanding loads beyond the vmcnt range");
  auto stage = [&](int s) -> char* { return s == 0 ? st0 : s == 1 ? st1 : s == 2 ? st2 : st3; };

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
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM;
  const int wn = wave / WM;

  // lane (r0, slot kc) of load group p fills slot kc of stacked row
  // r0 + p * RSTEP; rows of a thread differ by multiples of 16, so the
  // swizzle key, and the global chunk kc ^ key it loads, are per thread.
  constexpr unsigned OOB = 0x80000000u;
  const int r0 = tid >> 3;
  const int kc = tid & 7;
  const int gc = kc ^ (r0 & 6);
  const __amdgpu_buffer_rsrc_t rsA = __builtin_amdgcn_make_buffer_rsrc(
      (void*)g.A, (short)0, (int)((unsigned long long)g.M * g.lda * sizeof(T)), 0x00020000);
  const __amdgpu_buffer_rsrc_t rsB = __builtin_amdgcn_make_buffer_rsrc(
      (void*)g.B, (short)0, (int)((unsigned long long)g.N * g.ldb * sizeof(T)), 0x00020000);
  unsigned voff[CPT];
#pragma unroll
  for (int p = 0; p < CPT; ++p) {
    const int row = r0 + p * RSTEP;
    const unsigned kb = (unsigned)((kbeg + gc * VEC) * (int)sizeof(T));
    if (p * RSTEP < BM) {
      voff[p] = m0 + row < g.M ? (unsigned)((m0 + row) * (unsigned long long)g.lda * sizeof(T)) + kb : OOB;
    } else {
      voff[p] = n0 + row - BM < g.N ? (unsigned)((n0 + row - BM) * (unsigned long long)g.ldb * sizeof(T)) + kb
                                    : OOB;
    }
  }
  // K tile kt into LDS stage buffer dst: group p of this wave covers stacked
  // rows p * RSTEP + 8 * wave .. + 7 (a wave-uniform LDS address); the K
  // offset rides in the scalar offset.  A tile past the end (kt >= nk) is
  // still issued, with every lane's offset out of range: it moves no memory,
  // fills a stage that is never read again with zeros, and keeps the number
  // of loads per step fixed, so no branch surrounds a load and the wait
  // before each barrier is one constant.  (An offset of 2^31 or more stays
  // out of range whether or not the scalar offset is counted, and an
  // in-range row plus its K offset stays inside the operand.)
  auto dma = [&](int kt, char* dst) {
    const int kbytes = kt * BK * (int)sizeof(T);
    const unsigned past = kt < nk ? 0u : OOB;
#pragma unroll
    for (int p = 0; p < CPT; ++p) {
      const lds_ptr d = (lds_ptr)(dst + (p * RSTEP + 8 * wave) * ROWB);
      if (p * RSTEP < BM)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsA, d, 16, (int)(voff[p] | past), kbytes, 0, 0);
      else
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rsB, d, 16, (int)(voff[p] | past), kbytes, 0, 0);
    }
  };

  Acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  const int arow = wm * FM * 16 + (lane & 15);
  const int brow = BM + wn * FN * 16 + (lane & 15);
  const int swz_ld = lane & 6;
  const int kofs0 = (((lane >> 4) + 0) ^ swz_ld) * 16;
  const int kofs1 = (((lane >> 4) + 4) ^ swz_ld) * 16;
  auto compute = [&](const char* sb) {
#pragma unroll
    for (int kg = 0; kg < 2; ++kg) {
      uint4 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = *(const uint4*)(sb + (arow + i * 16) * ROWB + (kg ? kofs1 : kofs0));
#pragma unroll
      for (int j = 0; j < FN; ++j) bfr[j] = *(const uint4*)(sb + (brow + j * 16) * ROWB + (kg ? kofs1 : kofs0));
#pragma unroll
      for (int st = 0; st < Ops::STEPS; ++st)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) Ops::mma(acc[i][j], af[i], bfr[j], st);
    }
  };

  // prologue: tiles 0 .. NS-2 in flight
#pragma unroll
  for (int s = 0; s < NS - 1; ++s) dma(s, stage(s));
  // Tile k lives in stage k % NS.  Step k: wait for this wave's loads of
  // tile k (the NS-2 tiles issued after it stay in flight), barrier (every
  // wave's chunks of tile k landed; every wave finished reading tile k-1,
  // whose stage is refilled next), issue tile k+NS-1, multiply tile k.  The
  // loop body holds U steps (a multiple of NS, so every stage is a fixed
  // array in each step): the compiler's own wait before the first fragment
  // read after the loop head covers all earlier loads, which costs some
  // prefetch once per U tiles (larger U: more code and registers).  Issuing
  // the first tiles inside the loop instead avoids that wait but measured
  // 3 % (FP32) to 10 % (BF16) slower on the sweep shapes.
  if (nk > 0) {
    for (int kt = 0;; kt += U) {
#pragma unroll
      for (int s = 0; s < U; ++s) {
        wait_vm<(NS - 2) * CPT>();
        barrier_nofence();
        dma(kt + s + NS - 1, stage((s + NS - 1) % NS));
        compute(stage(s % NS));
        if (kt + s + 1 >= nk) goto done;
      }
    }
  }
done:
  wait_vm<0>();  // the trailing out-of-range loads

  const double acc64[1][1][4] = {};
  finish_tile<T, WM, WN, FM, FN, false, SWEEP>(g, acc, acc64, m0, n0, wm, wn, lane, split);
}

#define NNC_DMA_STAGES                                                            \
  constexpr int STAGE = dma_stage_bytes<T, WM, WN, FM, FN>();                     \
  __shared__ __attribute__((aligned(16))) char st0[STAGE];                        \
  __shared__ __attribute__((aligned(16))) char st1[STAGE];                        \
  __shared__ __attribute__((aligned(16))) char st2[NS > 2 ? STAGE : 16];          \
  __shared__ __attribute__((aligned(16))) char st3[NS > 3 ? STAGE : 16]

template <typename T, int WM, int WN, int FM, int FN, int NS, int U>
__global__ void __launch_bounds__(WM * WN * 64) gemm_dma_kernel(GemmArgs g) {
  NNC_DMA_STAGES;
  const int t = xcd_remap(blockIdx.x, gemm_tiles_per_split(g));
  dma_tile<T, WM, WN, FM, FN, NS, U, false>(g, t, blockIdx.y, st0, st1, st2, st3);
}

// Persistent grouped launch (several products; see gemm_grouped_kernel in
// gemm.hip): workgroup w takes work items w, w + gridDim.x, ...
template <typename T, int WM, int WN, int FM, int FN, int NS, int U>
__global__ void __launch_bounds__(WM * WN * 64)
gemm_grouped_dma_kernel(const GemmArgs* __restrict__ groups, const int* __restrict__ offsets, int ngroups) {
  NNC_DMA_STAGES;
  const int total = offsets[ngroups];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int gi = 0;
    while (gi + 1 < ngroups && offsets[gi + 1] <= w) ++gi;
    const GemmArgs g = groups[gi];
    const int local = w - offsets[gi];
    const int tiles = gemm_tiles_per_split(g);
    const int split = local / tiles;
    const int t = xcd_remap(local % tiles, tiles);
    dma_tile<T, WM, WN, FM, FN, NS, U, true>(g, t, split, st0, st1, st2, st3);
    __syncthreads();  // every wave done with the stages before the next item refills them
  }
}
#undef NNC_DMA_STAGES

template <typename T, int WM, int WN, int FM, int FN, int NS, int U>
static hipError_t launch_dma_cfg(GemmArgs g, int splits, hipStream_t s) {
  constexpr int BM = WM * FM * 16;
  constexpr int BN = WN * FN * 16;
  g.tiles_m = (g.M + BM - 1) / BM;
  g.tiles_n = (g.N + BN - 1) / BN;
  if (g.sym > 0 && (BM != g.sym || BN != g.sym || g.M != g.N)) return hipErrorInvalidValue;
  dim3 grid(gemm_tiles_per_split(g), splits);
  hipLaunchKernelGGL((gemm_dma_kernel<T, WM, WN, FM, FN, NS, U>), grid, dim3(WM * WN * 64), 0, s, g);
  return hipGetLastError();
}

template <typename T, int WM, int WN, int FM, int FN, int NS, int U>
static hipError_t launch_grouped_dma_cfg(const GemmArgs* groups, const int* offsets, int ngroups, int grid,
                                         hipStream_t s) {
  hipLaunchKernelGGL((gemm_grouped_dma_kernel<T, WM, WN, FM, FN, NS, U>), dim3(grid), dim3(WM * WN * 64), 0, s,
                     groups, offsets, ngroups);
  return hipGetLastError();
}

// FP32 and BF16 only: with FP64 operands the compiler adds a full wait
// before most fragment reads of this loop and the larger tiles spill.
// Variant = cfg - kFirstDmaCfg.
template <typename T, bool GROUPED>
static hipError_t launch_dma_typed(int variant, const GemmArgs& g, int splits, const GemmArgs* groups,
                                   const int* offsets, int ngroups, int grid, hipStream_t s) {
  switch (variant) {
    case 0:  // 128x128, 4 waves, 3 stages
      return GROUPED ? launch_grouped_dma_cfg<T, 2, 2, 4, 4, 3, 6>(groups, offsets, ngroups, grid, s)
                     : launch_dma_cfg<T, 2, 2, 4, 4, 3, 6>(g, splits, s);
    case 1:  // 128x256, 8 waves, 3 stages
      return GROUPED ? launch_grouped_dma_cfg<T, 2, 4, 4, 4, 3, 3>(groups, offsets, ngroups, grid, s)
                     : launch_dma_cfg<T, 2, 4, 4, 4, 3, 3>(g, splits, s);
    case 2:  // 64x64, 4 waves, 4 stages
      return GROUPED ? launch_grouped_dma_cfg<T, 2, 2, 2, 2, 4, 8>(groups, offsets, ngroups, grid, s)
                     : launch_dma_cfg<T, 2, 2, 2, 2, 4, 8>(g, splits, s);
    case 3:  // 64x64, 4 waves, 3 stages
      return GROUPED ? launch_grouped_dma_cfg<T, 2, 2, 2, 2, 3, 6>(groups, offsets, ngroups, grid, s)
                     : launch_dma_cfg<T, 2, 2, 2, 2, 3, 6>(g, splits, s);
    case 4:  // 128x128, 4 waves, 2 stages
      return GROUPED ? launch_grouped_dma_cfg<T, 2, 2, 4, 4, 2, 6>(groups, offsets, ngroups, grid, s)
                     : launch_dma_cfg<T, 2, 2, 4, 4, 2, 6>(g, splits, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_dma(DType t, int variant, GemmArgs g, int splits, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  switch (t) {
    case DT_F32: return launch_dma_typed<float, false>(variant, g, splits, nullptr, nullptr, 0, 0, s);
    case DT_BF16: return launch_dma_typed<bf16, false>(variant, g, splits, nullptr, nullptr, 0, 0, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_grouped_dma(DType t, int variant, const GemmArgs* groups, const int* offsets, int ngroups,
                                   int grid, hipStream_t s) {
  const GemmArgs none{};
  switch (t) {
    case DT_F32: return launch_dma_typed<float, true>(variant, none, 1, groups, offsets, ngroups, grid, s);
    case DT_BF16: return launch_dma_typed<bf16, true>(variant, none, 1, groups, offsets, ngroups, grid, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

// Workgroups of DMA tiling `variant` that fit on one CU (LDS-bound).
int gemm_dma_occupancy(int variant) {
  switch (variant) {
    case 2: case 4: return 2;   // 64 KB
    case 3: return 3;           // 48 KB
    default: return 1;          // 96 KB, 144 KB
  }
}

}  // namespace nnc
