// Device-side descriptors shared by the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "streamconv.h"

namespace sc {

// One stream's part of a processing step.  The runtime writes one Entry per
// stream into device memory before the step's launches.
struct Entry {
  const float* in;   // user input, channel-major [in_channels][T]
  float* out;        // user output, channel-major [out_channels][T * out_rate]
  float* state;      // the stream's state block (FP32, double-buffered regions)
  int32_t T;         // input frames in this buffer
  int32_t off;       // sum of T over the previous entries of the step
  int32_t parity;    // state copy holding the current caches (the other is written)
  int32_t flags;     // SC_FLAG_* of the stream
  int64_t pos;       // input frames processed before this buffer
  int64_t end;       // offline evaluation: input frames of the finite signal
                     // (every layer's output past its length is zeroed, the
                     // zero padding of Sec. 2.1 at the right edge); 0 = none
};

// Frames of `rate` (num/den per input frame) for t input frames (host side).
__host__ __device__ inline int64_t at_rate(int64_t t, int64_t num, int64_t den) { return t * num / den; }

// Unsigned 32-bit division by a run-time invariant d as a multiply-high, add
// and shift (Granlund & Montgomery, "Division by invariant integers using
// multiplication", 1994): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d)
// + 1, n / d = (mulhi(n, m) + n) >> l for every 32-bit n (the add is done in 64
// bits).  Device code never divides by a run-time value otherwise.
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.s = l;
  f.m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  return f;
}

__host__ __device__ inline uint32_t fdiv(const FastDiv& f, uint32_t n) {
  if (f.d == 1) return n;
#ifdef __HIP_DEVICE_COMPILE__
  const uint32_t t = __umulhi(n, f.m);
#else
  const uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
  return (uint32_t)(((uint64_t)t + n) >> f.s);
}

__device__ inline float lrelu(float v) { return v >= 0.f ? v : 0.2f * v; }

__device__ inline float sat448(float x) { return fminf(fmaxf(x, -448.f), 448.f); }

// One operand element: act(v) * qs rounded to the twin type, stored at
// element index `idx` of `base` (0 FP32, 1 BF16 RNE, 2 OCP FP8 e4m3 RNE saturating).
__device__ inline void store_twin1(void* base, int64_t idx, int prec, int pre, float qs, float v) {
  if (pre) v = lrelu(v);
  v *= qs;
  if (prec == 0) {
    static_cast<float*>(base)[idx] = v;
  } else if (prec == 1) {
    __bf16 h = (__bf16)v;
    static_cast<__bf16*>(base)[idx] = h;
  } else {
    const int q = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v), 0.f, 0, false);
    static_cast<unsigned char*>(base)[idx] = (unsigned char)(q & 0xff);
  }
}

// store_twin1 for 4 consecutive elements (idx a multiple of 4): the same
// conversions, one 16-, 8- or 4-byte store.
__device__ inline void store_twin4v(void* base, int64_t idx, int prec, int pre, float qs, float v0, float v1,
                                    float v2, float v3) {
  if (pre) {
    v0 = lrelu(v0);
    v1 = lrelu(v1);
    v2 = lrelu(v2);
    v3 = lrelu(v3);
  }
  v0 *= qs;
  v1 *= qs;
  v2 *= qs;
  v3 *= qs;
  if (prec == 0) {
    typedef float f4t __attribute__((ext_vector_type(4)));
    *reinterpret_cast<f4t*>(static_cast<float*>(base) + idx) = f4t{v0, v1, v2, v3};
  } else if (prec == 1) {
    typedef __bf16 b4t __attribute__((ext_vector_type(4)));
    *reinterpret_cast<b4t*>(static_cast<__bf16*>(base) + idx) = b4t{(__bf16)v0, (__bf16)v1, (__bf16)v2, (__bf16)v3};
  } else {
    int q = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v0), sat448(v1), 0, false);
    q = __builtin_amdgcn_cvt_pk_fp8_f32(sat448(v2), sat448(v3), q, true);
    *reinterpret_cast<int*>(static_cast<unsigned char*>(base) + idx) = q;
  }
}

}  // namespace sc
