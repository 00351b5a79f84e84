// Device-side helpers shared by the HIP kernels of libnnc (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16;

namespace nnc {

// ---------------------------------------------------------------- activations
// sigma, sigma', sigma'' of the smooth activations (Section 2 requires C^2).
// Evaluated in FP64 from z; tanh/exp/log1p come from the HIP device library.
enum Act { ACT_IDENTITY = 0, ACT_TANH = 1, ACT_SIGMOID = 2, ACT_SOFTPLUS = 3, ACT_SOFTMAX = 4 };

struct ActVal {
  double v, d1, d2;
};

__device__ __forceinline__ double sigmoid_d(double z) {
  // 1/(1+e^-z) without overflow for large |z|
  if (z >= 0.0) {
    return 1.0 / (1.0 + exp(-z));
  }
  double e = exp(z);
  return e / (1.0 + e);
}

__device__ __forceinline__ ActVal act_eval(int act, double z) {
  ActVal r;
  switch (act) {
    case ACT_TANH: {
      double t = tanh(z);
      double d = 1.0 - t * t;
      r.v = t;
      r.d1 = d;
      r.d2 = -2.0 * t * d;
      break;
    }
    case ACT_SIGMOID: {
      double s = sigmoid_d(z);
      double d = s * (1.0 - s);
      r.v = s;
      r.d1 = d;
      r.d2 = d * (1.0 - 2.0 * s);
      break;
    }
    case ACT_SOFTPLUS: {
      double s = sigmoid_d(z);
      r.v = (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
      r.d1 = s;
      r.d2 = s * (1.0 - s);
      break;
    }
    default:
      r.v = z;
      r.d1 = 1.0;
      r.d2 = 0.0;
  }
  return r;
}

// ---------------------------------------------------------------- conversions
template <typename T> __device__ __forceinline__ T from_f(float x);
template <> __device__ __forceinline__ float from_f<float>(float x) { return x; }
template <> __device__ __forceinline__ bf16 from_f<bf16>(float x) { return (bf16)x; }
template <> __device__ __forceinline__ double from_f<double>(float x) { return (double)x; }

template <typename T> __device__ __forceinline__ T from_d(double x);
template <> __device__ __forceinline__ float from_d<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ bf16 from_d<bf16>(double x) { return (bf16)(float)x; }
template <> __device__ __forceinline__ double from_d<double>(double x) { return x; }

template <typename T> __device__ __forceinline__ float to_f(T x) { return (float)x; }
template <typename T> __device__ __forceinline__ double to_d(T x) { return (double)(float)x; }
template <> __device__ __forceinline__ double to_d<double>(double x) { return x; }
template <> __device__ __forceinline__ double to_d<float>(float x) { return (double)x; }

// Store a value computed in accumulator type A into storage type T.
template <typename T, typename A> __device__ __forceinline__ T cvt_store(A x);
template <> __device__ __forceinline__ float cvt_store<float, float>(float x) { return x; }
template <> __device__ __forceinline__ bf16 cvt_store<bf16, float>(float x) { return (bf16)x; }
template <> __device__ __forceinline__ double cvt_store<double, double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_store<float, double>(double x) { return (float)x; }
template <> __device__ __forceinline__ double cvt_store<double, float>(float x) { return (double)x; }
template <> __device__ __forceinline__ bf16 cvt_store<bf16, double>(double x) { return (bf16)(float)x; }

// Unpack a 16-byte vector of storage type T into N accumulator-type values.
template <typename T, typename A> struct Vec16;
template <> struct Vec16<float, float> {
  static constexpr int N = 4;
  __device__ __forceinline__ static void unpack(const uint4& u, float* o) {
    o[0] = __uint_as_float(u.x);
    o[1] = __uint_as_float(u.y);
    o[2] = __uint_as_float(u.z);
    o[3] = __uint_as_float(u.w);
  }
};
template <> struct Vec16<float, double> {
  static constexpr int N = 4;
  __device__ __forceinline__ static void unpack(const uint4& u, double* o) {
    o[0] = __uint_as_float(u.x);
    o[1] = __uint_as_float(u.y);
    o[2] = __uint_as_float(u.z);
    o[3] = __uint_as_float(u.w);
  }
};
__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
template <> struct Vec16<bf16, float> {
  static constexpr int N = 8;
  __device__ __forceinline__ static void unpack(const uint4& u, float* o) {
    o[0] = bf16lo(u.x); o[1] = bf16hi(u.x);
    o[2] = bf16lo(u.y); o[3] = bf16hi(u.y);
    o[4] = bf16lo(u.z); o[5] = bf16hi(u.z);
    o[6] = bf16lo(u.w); o[7] = bf16hi(u.w);
  }
};
template <> struct Vec16<bf16, double> {
  static constexpr int N = 8;
  __device__ __forceinline__ static void unpack(const uint4& u, double* o) {
    o[0] = bf16lo(u.x); o[1] = bf16hi(u.x);
    o[2] = bf16lo(u.y); o[3] = bf16hi(u.y);
    o[4] = bf16lo(u.z); o[5] = bf16hi(u.z);
    o[6] = bf16lo(u.w); o[7] = bf16hi(u.w);
  }
};
template <> struct Vec16<double, double> {
  static constexpr int N = 2;
  __device__ __forceinline__ static void unpack(const uint4& u, double* o) {
    o[0] = __hiloint2double(u.y, u.x);
    o[1] = __hiloint2double(u.w, u.z);
  }
};

}  // namespace nnc
