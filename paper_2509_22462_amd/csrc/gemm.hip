// MFMA GEMM for gfx950 (CDNA4) with fused tangent-sweep epilogues: the
// tiling registry and the dispatch to the per-type instantiations
// (gemm_f32.hip, gemm_bf16.hip, gemm_f64.hip; the kernels and their design
// are described in gemm_kernels.h) and to the LDS-DMA-staged tilings from
// kFirstDmaCfg on (gemm_dma.hip, FP32 and BF16); the autotuner picks among
// all of them.
#include "gemm_common.h"

namespace nnc {

hipError_t gemm_launch_f32(int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s);
hipError_t gemm_launch_bf16(int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s);
hipError_t gemm_launch_f64(int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s);
hipError_t gemm_grouped_f32(int cfg, bool acc64, const GemmArgs* groups, const int* offsets, int ngroups, int grid,
                            hipStream_t s);
hipError_t gemm_grouped_bf16(int cfg, bool acc64, const GemmArgs* groups, const int* offsets, int ngroups, int grid,
                             hipStream_t s);
hipError_t gemm_grouped_f64(int cfg, bool acc64, const GemmArgs* groups, const int* offsets, int ngroups, int grid,
                            hipStream_t s);
hipError_t gemm_splitk_f32(GemmArgs g, const void* part, int splits, hipStream_t s);
hipError_t gemm_splitk_bf16(GemmArgs g, const void* part, int splits, hipStream_t s);
hipError_t gemm_splitk_f64(GemmArgs g, const void* part, int splits, hipStream_t s);

hipError_t launch_splitk_reduce(DType t, GemmArgs g, const void* part, int splits, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (splits < 1 || !part) return hipErrorInvalidValue;
  if (t == DT_F32) return gemm_splitk_f32(g, part, splits, s);
  if (t == DT_BF16) return gemm_splitk_bf16(g, part, splits, s);
  if (t == DT_F64) return gemm_splitk_f64(g, part, splits, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- registry
static const GemmCfg kCfgs[] = {
    {0, 128, 128, "128x128_w2x2"},
    {1, 208, 64, "208x64_w1x4"},
    {2, 208, 128, "208x128_w1x8"},
    {3, 64, 64, "64x64_w2x2"},
    {4, 256, 256, "256x256_w2x4"},
    {5, 112, 128, "112x128_w1x4"},
    {6, 128, 256, "128x256_w2x4"},
    {7, 112, 256, "112x256_w1x8"},
    // the same tilings with a two-tile prefetch
    {8, 128, 128, "128x128_w2x2_pf2"},
    {9, 208, 128, "208x128_w1x8_pf2"},
    {10, 112, 128, "112x128_w1x4_pf2"},
    {11, 112, 256, "112x256_w1x8_pf2"},
    {12, 256, 256, "256x256_w2x4_pf2"},
    {13, 128, 256, "128x256_w2x4_pf2"},
    // four waves with large wave tiles (fewer LDS bytes per MFMA)
    {14, 112, 256, "112x256_w1x4"},
    {15, 128, 256, "128x256_w2x2"},
    // LDS-DMA staging with 2 to 4 LDS stages (gemm_dma.hip)
    {16, 128, 128, "128x128_w2x2_dma3"},
    {17, 128, 256, "128x256_w2x4_dma3"},
    {18, 64, 64, "64x64_w2x2_dma4"},
    {19, 64, 64, "64x64_w2x2_dma3"},
    {20, 128, 128, "128x128_w2x2_dma2"},
};

int gemm_num_cfgs() { return (int)(sizeof(kCfgs) / sizeof(kCfgs[0])); }
const GemmCfg& gemm_cfg(int i) { return kCfgs[i]; }

bool gemm_grouped_supports(DType t, int cfg, bool acc64) {
  if (!gemm_cfg_supports(t, cfg, acc64)) return false;
  if (cfg == 0 || cfg == 1 || cfg == 3 || cfg == 5 || cfg >= kFirstDmaCfg) return true;
  return !acc64 && gemm_cfg_tunable(t, cfg) &&
         (cfg == 2 || cfg == 4 || cfg == 6 || cfg == 7 || cfg == 9 || cfg == 11 || cfg == 13);
}

// Workgroups of tiling cfg that fit on one CU together (LDS and registers),
// the per-CU width of a persistent grouped launch.
int gemm_grouped_occupancy(int cfg) {
  if (cfg >= kFirstDmaCfg) return gemm_dma_occupancy(cfg - kFirstDmaCfg);
  if (cfg == 3) return 4;
  if (cfg == 0 || cfg == 1 || cfg == 5) return 2;
  return 1;
}

void gemm_set_tiles(int cfg, GemmArgs& g) {
  const GemmCfg& c = kCfgs[cfg];
  g.tiles_m = (g.M + c.bm - 1) / c.bm;
  g.tiles_n = (g.N + c.bn - 1) / c.bn;
}

hipError_t launch_gemm_grouped(DType t, int cfg, bool acc64, const GemmArgs* groups, const int* offsets,
                               int ngroups, int grid, hipStream_t s) {
  if (!gemm_grouped_supports(t, cfg, acc64) || grid <= 0) return hipErrorInvalidValue;
  if (cfg >= kFirstDmaCfg) return launch_gemm_grouped_dma(t, cfg - kFirstDmaCfg, groups, offsets, ngroups, grid, s);
  switch (t) {
    case DT_F32: return gemm_grouped_f32(cfg, acc64, groups, offsets, ngroups, grid, s);
    case DT_BF16: return gemm_grouped_bf16(cfg, acc64, groups, offsets, ngroups, grid, s);
    case DT_F64: return gemm_grouped_f64(cfg, acc64, groups, offsets, ngroups, grid, s);
  }
  return hipErrorInvalidValue;
}

// Configurations the autotuner tries (the larger tiles that spill
// registers are kept out of the search).
bool gemm_cfg_tunable(DType t, int cfg) {
  if (cfg < 0 || cfg >= gemm_num_cfgs()) return false;
  // tilings that spill registers for that type (checked with the compiler's
  // resource report) stay out of the search
  if (t == DT_F64) return cfg != 2 && cfg != 4 && cfg != 9 && cfg != 11 && cfg != 12 && cfg != 13;
  if (t == DT_F32) return cfg != 4 && cfg != 12;
  return cfg != 12;
}

bool gemm_cfg_supports(DType t, int cfg, bool acc64) {
  if (cfg < 0 || cfg >= gemm_num_cfgs()) return false;
  if (acc64) {
    if (t == DT_F64) return false;  // FP64 MFMA already accumulates in FP64
    return cfg == 0 || cfg == 1 || cfg == 3;
  }
  return t != DT_F64 || cfg < kFirstDmaCfg;  // LDS-DMA tilings: FP32 and BF16
}

hipError_t launch_gemm(DType t, int cfg, bool acc64, GemmArgs g, int splits, hipStream_t s) {
  if (!gemm_cfg_supports(t, cfg, acc64)) return hipErrorInvalidValue;
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (cfg >= kFirstDmaCfg) return launch_gemm_dma(t, cfg - kFirstDmaCfg, g, splits, s);
  switch (t) {
    case DT_F32: return gemm_launch_f32(cfg, acc64, g, splits, s);
    case DT_BF16: return gemm_launch_bf16(cfg, acc64, g, splits, s);
    case DT_F64: return gemm_launch_f64(cfg, acc64, g, splits, s);
  }
  return hipErrorInvalidValue;
}


}  // namespace nnc
