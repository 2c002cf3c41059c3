// FP32 wavefront-FMA kernels: the narrow layers (few channels) and the
// FP32 path of any layer.  One lane per output value; consecutive lanes take
// consecutive output channels so that weight reads (packed [tap][cin][cout])
// coalesce and input reads broadcast.  Every sum is a fixed chain of fmaf in
// tap-major, channel-minor order that does not depend on where a frame sits
// in its buffer, so results are bitwise independent of the buffer split.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sc {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t items) {
  int64_t g = (items + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// Base pointer and channel stride of window row `row` of an entry: rows
// [0, L) are the cached previous input frames, rows >= L the new frames.
struct Row {
  const float* p;
  int64_t cs;
};

__device__ inline Row window_row(const LayerArgs& a, const Entry& e, int64_t in_start, int64_t Tin,
                                 int64_t row, int32_t L, int64_t soff, int64_t slen, const float* buf,
                                 int32_t C) {
  if (row < L) return Row{e.state + soff + (int64_t)e.parity * slen + row * C, 1};
  const int64_t r = row - L;
  if (buf) return Row{buf + (in_start + r) * C, 1};
  return Row{e.in + r, Tin};  // user input, channel-major
}

__global__ void __launch_bounds__(kBlock) conv_valu_kernel(LayerArgs a) {
  const int64_t n_items = a.n_out * a.cout;
  const int64_t per_ent = (int64_t)a.L * a.cin;
  const int64_t total = n_items + (int64_t)a.n_ent * per_ent;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    if (idx < n_items) {
      const int co = (int)(idx % a.cout);
      const int64_t n = idx / a.cout;
      const int ei = find_entry(a.ents, a.n_ent, n, a.out_num, a.out_den, 0);
      const Entry e = a.ents[ei];
      const int64_t out_start = at_rate(e.off, a.out_num, a.out_den);
      const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
      const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
      const int64_t t = n - out_start;
      const float* W = static_cast<const float*>(a.W);
      float acc = a.B[co];
      for (int kk = 0; kk < a.k; ++kk) {
        const Row rw = window_row(a, e, in_start, Tin, t * a.stride + (int64_t)a.dil * kk, a.L,
                                  a.state_off, a.state_len, a.in_buf, a.cin);
        const float* wp = W + (int64_t)kk * a.cin * a.cout + co;
        if (a.pre_act) {
          for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], lrelu(rw.p[ci * rw.cs]), acc);
        } else {
          for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], rw.p[ci * rw.cs], acc);
        }
      }
      if (a.residual) {
        const Row rw = window_row(a, e, in_start, Tin, t + a.skip_off, a.L, a.state_off, a.state_len,
                                  a.in_buf, a.cin);
        acc = acc + rw.p[co * rw.cs];
      }
      if (a.post_act == 2) acc = tanhf(acc);
      if ((e.flags & SC_FLAG_WARMUP_MASK) && at_rate(e.pos, a.out_num, a.out_den) + t < a.delay) acc = 0.f;
      if (a.out_buf) {
        a.out_buf[n * a.cout + co] = acc;
      } else {
        const int64_t Tout = at_rate(e.T, a.out_num, a.out_den);
        e.out[(int64_t)co * Tout + t] = acc;
      }
    } else {
      // cache update: new cache = window rows [Tin, Tin + L) into the other copy
      const int64_t j = idx - n_items;
      const int ei = (int)(j / per_ent);
      const int64_t rem = j % per_ent;
      const int64_t i = rem / a.cin;
      const int ci = (int)(rem % a.cin);
      const Entry e = a.ents[ei];
      const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
      const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
      const Row rw = window_row(a, e, in_start, Tin, Tin + i, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
      e.state[a.state_off + (int64_t)(1 - e.parity) * a.state_len + i * a.cin + ci] = rw.p[ci * rw.cs];
    }
  }
}

// Transposed conv, kernel 2r: output frame q*r + phi of a buffer is
//   W[phi + r] . a[q-1] + W[phi] . a[q]   (+ bias),
// accumulated in that order.  Column q = T of each entry holds only the
// first half: it is the FP32 overlap carry that column q = 0 of the next
// buffer starts from, so the chain of fmaf is the same for every frame.
// Weights packed [h][phi][cin][cout], h = 0 -> tap phi + r, h = 1 -> tap phi.
__global__ void __launch_bounds__(kBlock) convt_valu_kernel(LayerArgs a) {
  const int r = a.stride;
  const int64_t n_cols = a.n_in + a.n_ent;
  const int64_t total = n_cols * r * a.cout;
  const float* W = static_cast<const float*>(a.W);
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    const int co = (int)(idx % a.cout);
    const int64_t rest = idx / a.cout;
    const int phi = (int)(rest % r);
    const int64_t c = rest / r;
    const int ei = find_entry(a.ents, a.n_ent, c, a.in_num, a.in_den, 1);
    const Entry e = a.ents[ei];
    const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
    const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
    const int64_t q = c - in_start - ei;
    const float* carry_in = e.state + a.state_off + (int64_t)e.parity * a.state_len;
    float acc = (q == 0) ? carry_in[phi * a.cout + co] : 0.f;
    for (int h = 0; h < 2; ++h) {
      const int64_t row = q - 1 + h;
      if (row < 0 || row >= Tin) continue;
      const float* x = a.in_buf ? a.in_buf + (in_start + row) * a.cin : e.in + row;
      const int64_t xs = a.in_buf ? 1 : Tin;
      const float* wp = W + ((int64_t)(h * r + phi) * a.cin) * a.cout + co;
      if (a.pre_act) {
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], lrelu(x[ci * xs]), acc);
      } else {
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], x[ci * xs], acc);
      }
    }
    if (q < Tin) {
      float v = acc + a.B[co];
      const int64_t t = q * r + phi;
      if ((e.flags & SC_FLAG_WARMUP_MASK) && at_rate(e.pos, a.out_num, a.out_den) + t < a.delay) v = 0.f;
      if (a.out_buf) {
        a.out_buf[(in_start * r + t) * a.cout + co] = v;
      } else {
        e.out[(int64_t)co * (Tin * r) + t] = v;
      }
    } else {
      e.state[a.state_off + (int64_t)(1 - e.parity) * a.state_len + phi * a.cout + co] = acc;
    }
  }
}

// Sum of two branches, branch j delayed by A_j frames through a delay line
// (Eq. 3).  Window of branch j: [line_j (A_j frames) | new frames].
__global__ void __launch_bounds__(kBlock) delay_add_kernel(LayerArgs a) {
  const int C = a.cout;
  const int64_t n_items = a.n_out * C;
  const int64_t per_ent = (int64_t)(a.A0 + a.A1) * C;
  const int64_t total = n_items + (int64_t)a.n_ent * per_ent;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    if (idx < n_items) {
      const int c = (int)(idx % C);
      const int64_t n = idx / C;
      const int ei = find_entry(a.ents, a.n_ent, n, a.out_num, a.out_den, 0);
      const Entry e = a.ents[ei];
      const int64_t start = at_rate(e.off, a.out_num, a.out_den);
      const int64_t Tn = at_rate(e.T, a.out_num, a.out_den);
      const int64_t t = n - start;
      const Row r0 = window_row(a, e, start, Tn, t, a.A0, a.state_off, a.state_len, a.in_buf, C);
      const Row r1 = window_row(a, e, start, Tn, t, a.A1, a.state_off2, a.state_len2, a.in_buf2, C);
      float v = r0.p[c * r0.cs] + r1.p[c * r1.cs];
      if ((e.flags & SC_FLAG_WARMUP_MASK) && at_rate(e.pos, a.out_num, a.out_den) + t < a.delay) v = 0.f;
      if (a.out_buf) a.out_buf[n * C + c] = v;
      else e.out[(int64_t)c * Tn + t] = v;
    } else {
      const int64_t j = idx - n_items;
      const int ei = (int)(j / per_ent);
      int64_t rem = j % per_ent;
      const Entry e = a.ents[ei];
      const int64_t start = at_rate(e.off, a.out_num, a.out_den);
      const int64_t Tn = at_rate(e.T, a.out_num, a.out_den);
      const bool second = rem >= (int64_t)a.A0 * C;
      if (second) rem -= (int64_t)a.A0 * C;
      const int64_t i = rem / C;
      const int c = (int)(rem % C);
      const int32_t A = second ? a.A1 : a.A0;
      const int64_t soff = second ? a.state_off2 : a.state_off;
      const int64_t slen = second ? a.state_len2 : a.state_len;
      const Row rw = window_row(a, e, start, Tn, Tn + i, A, soff, slen, second ? a.in_buf2 : a.in_buf, C);
      e.state[soff + (int64_t)(1 - e.parity) * slen + i * C + c] = rw.p[c * rw.cs];
    }
  }
}

__global__ void __launch_bounds__(kBlock) amax_kernel(LayerArgs a, float* amax) {
  __shared__ float red[kBlock];
  float m = 0.f;
  const int64_t total = a.n_in * a.cin;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    float v;
    if (a.in_buf) {
      v = a.in_buf[idx];
    } else {
      const int ci = (int)(idx % a.cin);
      const int64_t n = idx / a.cin;
      const int ei = find_entry(a.ents, a.n_ent, n, a.in_num, a.in_den, 0);
      const Entry e = a.ents[ei];
      const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
      v = e.in[(int64_t)ci * Tin + (n - at_rate(e.off, a.in_num, a.in_den))];
    }
    if (a.pre_act) v = lrelu(v);
    m = fmaxf(m, fabsf(v));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(reinterpret_cast<unsigned int*>(amax), __float_as_uint(red[0]));
}

__global__ void __launch_bounds__(kBlock) fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.f;
}

}  // namespace

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_conv_valu(const LayerArgs& a, hipStream_t s) {
  const int64_t items = a.n_out * a.cout + (int64_t)a.n_ent * a.L * a.cin;
  hipLaunchKernelGGL(conv_valu_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_convt_valu(const LayerArgs& a, hipStream_t s) {
  const int64_t items = (a.n_in + a.n_ent) * a.stride * a.cout;
  hipLaunchKernelGGL(convt_valu_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_delay_add(const LayerArgs& a, hipStream_t s) {
  const int64_t items = a.n_out * a.cout + (int64_t)a.n_ent * (a.A0 + a.A1) * a.cout;
  hipLaunchKernelGGL(delay_add_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_amax(const LayerArgs& a, float* amax, hipStream_t s) {
  const int64_t items = a.n_in * a.cin;
  int g = grid_for(items);
  if (g > 1024) g = 1024;
  hipLaunchKernelGGL(amax_kernel, dim3(g), dim3(kBlock), 0, s, a, amax);
  return hipGetLastError();
}

}  // namespace sc
