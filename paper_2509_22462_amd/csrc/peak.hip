// Peak microbenchmarks: the MFMA issue rate and the HBM stream rate that
// plain loops reach on this GPU.  They are the measured ceilings beside the
// datasheet peaks against which the library's MFMA-bound kernels (the
// tangent-sweep and H products) and HBM-bound kernels (the weight streams)
// are read.
//
//   * peak_mfma_kernel: every wave runs 8 (4 for the 32x32 shape) independent
//     accumulator chains of one MFMA shape from registers (no memory traffic in the
//     loop), 16 waves per CU, so the matrix pipes never wait on a dependency.
//   * peak_read_kernel / peak_copy_kernel: grid-stride 16-byte loads (and
//     stores), four in flight per thread, over a caller buffer that should
//     exceed the 256 MB Infinity Cache so that HBM, not the cache, is timed.
#include <algorithm>

#include "nnc.h"
#include "nnc_device.h"
#include "nnc_internal.h"

namespace nnc {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kChains = 8;       // independent accumulator chains per wave (16x16 shapes)
constexpr int kChains32 = 4;     // (32x32 shape: 16 accumulator registers each)
constexpr int kPeakThreads = 256;
constexpr int kMfmaBlocksPerCU = 4;

// Flops of one MFMA of each kind (2 * M * N * K).
constexpr double kMfmaFlops[NNC_PEAK_NKINDS] = {2.0 * 16 * 16 * 32, 2.0 * 32 * 32 * 16, 2.0 * 16 * 16 * 4,
                                                 2.0 * 16 * 16 * 4};

// Four waves per SIMD (the launch's 16 per CU): with that register budget
// the compiler keeps each chain's accumulator in place across iterations
// (with a larger budget it moves them between register files every
// iteration, and the loop no longer measures the MFMA rate).
template <int KIND>
__global__ void __launch_bounds__(kPeakThreads) __attribute__((amdgpu_waves_per_eu(4)))
peak_mfma_kernel(int iters, float* sink) {
  const int lane = threadIdx.x & 63;
  float s = 0.0f;
  if constexpr (KIND == NNC_PEAK_BF16_16X16X32 || KIND == NNC_PEAK_BF16_32X32X16) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (bf16)(1e-3f * (float)(lane + e));
      b[e] = (bf16)(1e-3f * (float)(lane - e));
    }
    if constexpr (KIND == NNC_PEAK_BF16_16X16X32) {
      floatx4 acc[kChains];
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = floatx4{0, 0, 0, 0};
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
#pragma unroll
      for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    } else {
      floatx16 acc[kChains32];
#pragma unroll
      for (int c = 0; c < kChains32; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[c][e] = 0.0f;
      for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int c = 0; c < kChains32; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
#pragma unroll
      for (int c = 0; c < kChains32; ++c)
#pragma unroll
        for (int e = 0; e < 16; ++e) s += acc[c][e];
    }
  } else if constexpr (KIND == NNC_PEAK_FP32_16X16X4) {
    const float a = 1e-3f * (float)lane, b = 1e-3f * (float)(64 - lane);
    floatx4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = floatx4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else {
    const double a = 1e-3 * (double)lane, b = 1e-3 * (double)(64 - lane);
    doublex4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = doublex4{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    double d = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) d += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    s = (float)d;
  }
  sink[(size_t)blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// Reads n 16-byte words; the XOR of everything read decides a store that
// keeps the loads alive (dst holds at least one word).
__global__ void __launch_bounds__(kPeakThreads) peak_read_kernel(const uint4* __restrict__ src, size_t n,
                                                                  uint4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x;
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    acc.x ^= v0.x ^ v1.x ^ v2.x ^ v3.x;
    acc.y ^= v0.y ^ v1.y ^ v2.y ^ v3.y;
    acc.z ^= v0.z ^ v1.z ^ v2.z ^ v3.z;
    acc.w ^= v0.w ^ v1.w ^ v2.w ^ v3.w;
  }
  for (; i < n; i += stride) {
    const uint4 v = src[i];
    acc.x ^= v.x;
    acc.y ^= v.y;
    acc.z ^= v.z;
    acc.w ^= v.w;
  }
  if ((acc.x & acc.y & acc.z & acc.w) == 0xFFFFFFFFu) dst[0] = acc;
}

__global__ void __launch_bounds__(kPeakThreads) peak_copy_kernel(const uint4* __restrict__ src, size_t n,
                                                                  uint4* __restrict__ dst) {
  const size_t stride = (size_t)gridDim.x * kPeakThreads;
  size_t i = (size_t)blockIdx.x * kPeakThreads + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
    dst[i] = v0;
    dst[i + stride] = v1;
    dst[i + 2 * stride] = v2;
    dst[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

template <int KIND>
hipError_t launch_peak_mfma(int blocks, int iters, float* sink, hipStream_t s) {
  hipLaunchKernelGGL(peak_mfma_kernel<KIND>, dim3(blocks), dim3(kPeakThreads), 0, s, iters, sink);
  return hipGetLastError();
}

hipError_t launch_peak_mfma_kind(int kind, int blocks, int iters, float* sink, hipStream_t s) {
  switch (kind) {
    case NNC_PEAK_BF16_16X16X32: return launch_peak_mfma<NNC_PEAK_BF16_16X16X32>(blocks, iters, sink, s);
    case NNC_PEAK_BF16_32X32X16: return launch_peak_mfma<NNC_PEAK_BF16_32X32X16>(blocks, iters, sink, s);
    case NNC_PEAK_FP32_16X16X4: return launch_peak_mfma<NNC_PEAK_FP32_16X16X4>(blocks, iters, sink, s);
    case NNC_PEAK_FP64_16X16X4: return launch_peak_mfma<NNC_PEAK_FP64_16X16X4>(blocks, iters, sink, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

int fail(Ctx* c, int code, const std::string& msg) {
  c->err = msg;
  return code;
}

// Milliseconds between two events recorded around `launch` on stream s.
template <typename F>
hipError_t time_on_stream(hipStream_t s, F launch, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  return e;
}

}  // namespace
}  // namespace nnc

using namespace nnc;

extern "C" {

int nnc_peak_mfma(nnc_ctx ctx, int kind, int iters, double* tflops) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (kind < 0 || kind >= NNC_PEAK_NKINDS) return fail(c, NNC_E_ARG, "unknown MFMA kind");
  if (iters < 1 || iters > (1 << 22)) return fail(c, NNC_E_SHAPE, "iters outside 1 .. 2^22");
  if (!tflops) return fail(c, NNC_E_ARG, "null tflops");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NNC_E_HIP, "hipSetDevice failed");
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
    return fail(c, NNC_E_HIP, "hipDeviceGetAttribute (compute units) failed");
  const int blocks = cus * kMfmaBlocksPerCU;
  float* sink = nullptr;
  if (hipMalloc(&sink, (size_t)blocks * kPeakThreads * sizeof(float)) != hipSuccess)
    return fail(c, NNC_E_NOMEM, "hipMalloc of the probe's sink failed");
  hipError_t e = launch_peak_mfma_kind(kind, blocks, iters, sink, c->stream);  // warm-up
  float ms = 0.0f;
  if (e == hipSuccess)
    e = time_on_stream(c->stream, [&] { return launch_peak_mfma_kind(kind, blocks, iters, sink, c->stream); }, &ms);
  hipFree(sink);
  if (e != hipSuccess) return fail(c, NNC_E_HIP, std::string("MFMA peak probe: ") + hipGetErrorString(e));
  const double waves = (double)blocks * (kPeakThreads / 64);
  const int chains = kind == NNC_PEAK_BF16_32X32X16 ? kChains32 : kChains;
  *tflops = waves * iters * chains * kMfmaFlops[kind] / (ms * 1e-3) / 1e12;
  return NNC_OK;
}

int nnc_peak_hbm(nnc_ctx ctx, const void* src, void* dst, size_t bytes, int reps, double* read_gbs,
                 double* copy_gbs) {
  Ctx* c = (Ctx*)ctx;
  if (!c) return NNC_E_ARG;
  if (!src || !dst) return fail(c, NNC_E_ARG, "null src or dst");
  if (!read_gbs && !copy_gbs) return fail(c, NNC_E_ARG, "no output requested");
  if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return fail(c, NNC_E_ARG, "src and dst must be 16-byte aligned");
  if (bytes < 16 || bytes % 16 != 0) return fail(c, NNC_E_SHAPE, "bytes must be a positive multiple of 16");
  if (reps < 1 || reps > 1000) return fail(c, NNC_E_SHAPE, "reps outside 1 .. 1000");
  const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
  if (copy_gbs && s0 < d0 + bytes && d0 < s0 + bytes) return fail(c, NNC_E_ARG, "src and dst overlap");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, NNC_E_HIP, "hipSetDevice failed");
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
    return fail(c, NNC_E_HIP, "hipDeviceGetAttribute (compute units) failed");
  const size_t n = bytes / 16;
  const size_t want = (n + kPeakThreads - 1) / kPeakThreads;
  const int blocks = (int)std::min<size_t>((size_t)cus * 8, want);
  const uint4* s = (const uint4*)src;
  uint4* d = (uint4*)dst;
  auto read = [&] {
    for (int r = 0; r < reps; ++r) {
      hipLaunchKernelGGL(peak_read_kernel, dim3(blocks), dim3(kPeakThreads), 0, c->stream, s, n, d);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto copy = [&] {
    for (int r = 0; r < reps; ++r) {
      hipLaunchKernelGGL(peak_copy_kernel, dim3(blocks), dim3(kPeakThreads), 0, c->stream, s, n, d);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  float ms = 0.0f;
  if (read_gbs) {
    hipLaunchKernelGGL(peak_read_kernel, dim3(blocks), dim3(kPeakThreads), 0, c->stream, s, n, d);  // warm-up
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = time_on_stream(c->stream, read, &ms);
    if (e != hipSuccess) return fail(c, NNC_E_HIP, std::string("HBM read probe: ") + hipGetErrorString(e));
    *read_gbs = (double)bytes * reps / (ms * 1e-3) / 1e9;
  }
  if (copy_gbs) {
    hipLaunchKernelGGL(peak_copy_kernel, dim3(blocks), dim3(kPeakThreads), 0, c->stream, s, n, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = time_on_stream(c->stream, copy, &ms);
    if (e != hipSuccess) return fail(c, NNC_E_HIP, std::string("HBM copy probe: ") + hipGetErrorString(e));
    *copy_gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
  }
  return NNC_OK;
}

}  // extern "C"
