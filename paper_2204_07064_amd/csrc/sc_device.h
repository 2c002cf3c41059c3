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
};

// Frames of `rate` (num/den per input frame) for t input frames.
__device__ __host__ inline int64_t at_rate(int64_t t, int64_t num, int64_t den) { return t * num / den; }

// Entry of packed frame n at rate num/den: fent maps every input frame of the
// step to its entry, and frame n of a layer lies in input frame n * den / num.
__device__ inline int entry_at(const int32_t* fent, int64_t n, int64_t num, int64_t den) {
  return fent[n * den / num];
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

}  // namespace sc
