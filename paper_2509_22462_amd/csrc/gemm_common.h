// Device code shared by the MFMA GEMM kernels (gemm.hip: register-staged
// tiles; gemm_dma.hip: LDS-DMA-staged tiles): MFMA wrappers and their
// accumulator layouts, the fused epilogues, tile stores and the XCD-aware
// tile order.
#pragma once
#include "nnc_device.h"
#include "nnc_internal.h"

namespace nnc {

template <typename T> struct MfmaOps;

// Output layout of the 16x16 accumulator: register e of lane l holds
// D[row_in_block(l, e)][l % 16].  fp32 and bf16: row 4*(l/16) + e;
// fp64 (v_mfma_f64_16x16x4): row l/16 + 4*e (checked on gfx950).
template <> struct MfmaOps<float> {
  using Acc = floatx4;
  using AccT = float;
  using AT = float;  // per-point vector type (sigma')
  __device__ __forceinline__ static int row_in_block(int lane, int e) { return (lane >> 4) * 4 + e; }
  static constexpr int STEPS = 4;  // MFMAs per 16-byte fragment pair
  __device__ __forceinline__ static void mma(Acc& c, const uint4& a, const uint4& b, int s) {
    const uint32_t av = s == 0 ? a.x : s == 1 ? a.y : s == 2 ? a.z : a.w;
    const uint32_t bv = s == 0 ? b.x : s == 1 ? b.y : s == 2 ? b.z : b.w;
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(av), __uint_as_float(bv), c, 0, 0, 0);
  }
};

template <> struct MfmaOps<bf16> {
  using Acc = floatx4;
  using AccT = float;
  using AT = float;
  __device__ __forceinline__ static int row_in_block(int lane, int e) { return (lane >> 4) * 4 + e; }
  static constexpr int STEPS = 1;
  __device__ __forceinline__ static void mma(Acc& c, const uint4& a, const uint4& b, int) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};

template <> struct MfmaOps<double> {
  using Acc = doublex4;
  using AccT = double;
  using AT = double;
  __device__ __forceinline__ static int row_in_block(int lane, int e) { return (lane >> 4) + 4 * e; }
  static constexpr int STEPS = 2;
  __device__ __forceinline__ static void mma(Acc& c, const uint4& a, const uint4& b, int s) {
    const double av = s == 0 ? __hiloint2double(a.y, a.x) : __hiloint2double(a.w, a.z);
    const double bv = s == 0 ? __hiloint2double(b.y, b.x) : __hiloint2double(b.w, b.z);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
  }
};

// Fused epilogue for one output element (mode EPI, compile time).  V is
// float or double.
template <typename T, typename V, int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, int row, int col, V v, int split) {
  using AT = typename MfmaOps<T>::AT;
  const long long o = (long long)row * g.ldo + col;
  switch (EPI) {
    case EPI_FWD_T: {
      const int b = row / g.rdiv;
      const V d1 = (V)((const AT*)g.v0)[(long long)b * g.ldv + col];
      ((T*)g.out0)[o] = cvt_store<T>(v);
      ((T*)g.out1)[o] = cvt_store<T>(v * d1);
      break;
    }
    case EPI_FWD_G: {
      const int b = row / g.rdiv;
      const V sv = (V)((const double*)g.v0)[(long long)b * g.ldv + col];
      ((T*)g.out0)[o] = cvt_store<T>(v * sv);
      break;
    }
    case EPI_REV_G: {
      const int b = row / g.rdiv;
      const long long vi = (long long)b * g.ldv + col;
      const V d1 = (V)((const AT*)g.v0)[vi];
      const V sv = (V)((const double*)g.v1)[vi];
      const int r2 = g.auxmod > 0 ? row % g.auxmod : row;
      const V tv = (V)to_d(((const T*)g.aux)[(long long)r2 * g.ldaux + col]);
      ((T*)g.out0)[o] = cvt_store<T>(d1 * v + sv * tv);
      break;
    }
    case EPI_FWD_LS: {
      const int b = row / g.rdiv;
      const long long vi = (long long)b * g.ldv + col;
      const V sv = (V)((const double*)g.v1)[vi];
      ((T*)g.out0)[o] = cvt_store<T>(v);
      ((T*)g.out2)[o] = cvt_store<T>(v * sv);
      if (g.out1) {
        const V d1 = (V)((const AT*)g.v0)[vi];
        ((T*)g.out1)[(long long)row * g.ldo1 + col] = cvt_store<T>(v * d1);
      }
      break;
    }
    case EPI_FWD_LT: {
      ((T*)g.out0)[o] = cvt_store<T>(v);
      if (g.out1) {
        const V d1 = (V)((const AT*)g.v0)[(long long)(row / g.rdiv) * g.ldv + col];
        ((T*)g.out1)[(long long)row * g.ldo1 + col] = cvt_store<T>(v * d1);
      }
      break;
    }
    case EPI_H64:
      ((double*)g.out0)[(long long)split * g.split_stride + o] = (double)v;
      break;
    case EPI_JAC_R: {
      const int b = row / g.rdiv;
      const V d1 = (V)((const AT*)g.v0)[(long long)b * g.ldv + col];
      ((AT*)g.out0)[o] = (AT)(v * d1);
      break;
    }
    case EPI_F64:
      ((double*)g.out0)[o] = (double)v;
      break;
    case EPI_TRAIN_FWD: {
      const float z = (float)v + g.bias[col];
      if (g.act == ACT_TANH) {
        const float a = tanhf(z);
        ((T*)g.out0)[o] = cvt_store<T>((V)a);
        ((T*)g.out1)[(long long)col * g.ldt + row] = cvt_store<T>((V)a);
        ((float*)g.out2)[o] = 1.0f - a * a;
      } else {
        ((float*)g.out2)[o] = z;
      }
      break;
    }
    case EPI_TRAIN_BWD: {
      const float dz = (float)v * ((const float*)g.v0)[(long long)row * g.ldv + col];
      ((T*)g.out0)[o] = cvt_store<T>((V)dz);
      ((T*)g.out1)[(long long)col * g.ldt + row] = cvt_store<T>((V)dz);
      break;
    }
    case EPI_F32:
      ((float*)g.out0)[o] = (float)v;
      break;
    case EPI_PART:
      ((float*)g.out0)[(long long)split * g.split_stride + o] = (float)v;
      break;
    case EPI_PART64:
      ((double*)g.out0)[(long long)split * g.split_stride + o] = (double)v;
      break;
    case EPI_PRIMAL: {
      double z = 0.0;
      ActVal av{0.0, 0.0, 0.0};
      if (col < g.dtrue) {
        z = (double)v + g.bias64[col];
        av = act_eval(g.act, z);
      }
      ((double*)g.out0)[o] = z;
      ((AT*)g.out1)[o] = (AT)av.v;
      ((AT*)g.out2)[o] = (AT)av.d1;
      break;
    }
    case EPI_ADJ64: {
      double zb = 0.0, sv = 0.0;
      if (col < g.dtrue) {
        const ActVal av = act_eval(g.act, ((const double*)g.v0)[(long long)row * g.ldv + col]);
        zb = (double)v * av.d1;
        sv = (double)v * av.d2;
      }
      ((double*)g.out0)[o] = zb;
      ((double*)g.out1)[o] = sv;
      break;
    }
    default:
      ((T*)g.out0)[o] = cvt_store<T>(v);
  }
}

// Store a finished tile through epilogue EPI; the (i, j, e) loops unroll
// fully, so accumulators stay in registers.
template <typename T, int WM, int WN, int FM, int FN, int EPI, typename Get>
__device__ __forceinline__ void store_tile(const GemmArgs& g, Get get, int m0, int n0, int wm, int wn,
                                           int lane, int split) {
  using Ops = MfmaOps<T>;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + wn * FN * 16 + j * 16 + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * FM * 16 + i * 16 + Ops::row_in_block(lane, e);
        if (row < g.M && col < g.N) {
          const auto v = get(i, j, e);
          gemm_epilogue<T, decltype(v), EPI>(g, row, col, v, split);
        }
      }
    }
  }
}

template <typename T, int WM, int WN, int FM, int FN>
struct TileShape {
  static constexpr int NT = WM * WN * 64;
  static constexpr int BM = WM * FM * 16;
  static constexpr int BN = WN * FN * 16;
  static constexpr int ROWB = 128;  // LDS row pitch (bytes), XOR-swizzled chunks
  static constexpr int STAGE = (BM + BN) * ROWB;
  static constexpr int SMEM = 2 * STAGE;
};

// Tile t of one K split -> (tm, tn) of its product.  Batched products
// (nbat > 0) point g at product b's operands and output first; symmetric ones
// (sym > 0) enumerate the lower block triangle row by row: t -> (tm, tn)
// with tm (tm + 1) / 2 <= t < (tm + 1) (tm + 2) / 2, tn = t - tm (tm + 1) / 2.
template <typename T>
__device__ __forceinline__ void locate_tile(GemmArgs& g, int t, int& tm, int& tn) {
  if (g.nbat > 0) {
    const int per = g.sym > 0 ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
    const int b = t / per;
    t -= b * per;
    g.A = (const T*)g.A + b * g.bsA;
    g.B = (const T*)g.B + b * g.bsB;
    g.out0 = (double*)g.out0 + b * g.bsO;
  }
  if (g.sym > 0) {
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (r > 0 && r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    tm = r;
    tn = t - r * (r + 1) / 2;
  } else {
    tm = t % g.tiles_m;
    tn = t / g.tiles_m;
  }
}

// XCD-aware permutation of tile ids: workgroup ids are dispatched to the 8
// XCDs round-robin; give each XCD a contiguous run of tile ids (tiles with
// consecutive ids share the same weight tile), bijective on [0, tiles).
__device__ __forceinline__ int xcd_remap(int t, int tiles) {
  const int full = tiles - tiles % 8;
  return t < full ? (t % 8) * (full / 8) + t / 8 : t;
}

// Epilogue of a finished tile: lane holds column lane%16 of each block, rows
// per MfmaOps::row_in_block; one specialised store loop per epilogue mode.
// SWEEP builds only the tangent-sweep epilogues (grouped launches).
template <typename T, int WM, int WN, int FM, int FN, bool ACC64, bool SWEEP, typename Acc, int A1, int A2>
__device__ __forceinline__ void finish_tile(const GemmArgs& g, const Acc (&acc)[FM][FN], const double (&acc64)[A1][A2][4],
                                            int m0, int n0, int wm, int wn, int lane, int split) {
  if constexpr (ACC64) {
    auto get = [&](int i, int j, int e) { return acc64[i][j][e]; };
    store_tile<T, WM, WN, FM, FN, EPI_H64>(g, get, m0, n0, wm, wn, lane, split);
  } else {
    auto get = [&](int i, int j, int e) { return acc[i][j][e]; };
#define NNC_STORE(E) store_tile<T, WM, WN, FM, FN, E>(g, get, m0, n0, wm, wn, lane, split)
    if constexpr (SWEEP) {  // tangent-sweep products only (grouped launches)
      switch (g.epi) {
        case EPI_FWD_T: NNC_STORE(EPI_FWD_T); break;
        case EPI_FWD_G: NNC_STORE(EPI_FWD_G); break;
        case EPI_REV_G: NNC_STORE(EPI_REV_G); break;
        case EPI_FWD_LS: NNC_STORE(EPI_FWD_LS); break;
        case EPI_H64: NNC_STORE(EPI_H64); break;
        case EPI_PART: NNC_STORE(EPI_PART); break;
        case EPI_PART64: NNC_STORE(EPI_PART64); break;
        default: break;
      }
      return;
    }
    switch (g.epi) {
      case EPI_FWD_T: NNC_STORE(EPI_FWD_T); break;
      case EPI_FWD_G: NNC_STORE(EPI_FWD_G); break;
      case EPI_REV_G: NNC_STORE(EPI_REV_G); break;
      case EPI_FWD_LS: NNC_STORE(EPI_FWD_LS); break;
      case EPI_FWD_LT: NNC_STORE(EPI_FWD_LT); break;
      case EPI_H64: NNC_STORE(EPI_H64); break;
      case EPI_JAC_R: NNC_STORE(EPI_JAC_R); break;
      case EPI_F64: NNC_STORE(EPI_F64); break;
      case EPI_TRAIN_FWD: NNC_STORE(EPI_TRAIN_FWD); break;
      case EPI_TRAIN_BWD: NNC_STORE(EPI_TRAIN_BWD); break;
      case EPI_F32: NNC_STORE(EPI_F32); break;
      case EPI_PART: NNC_STORE(EPI_PART); break;
      case EPI_PART64: NNC_STORE(EPI_PART64); break;
      case EPI_PRIMAL: NNC_STORE(EPI_PRIMAL); break;
      case EPI_ADJ64:
        if constexpr (sizeof(T) == 8) NNC_STORE(EPI_ADJ64);
        break;
      default: NNC_STORE(EPI_PLAIN); break;
    }
#undef NNC_STORE
  }
}

}  // namespace nnc
