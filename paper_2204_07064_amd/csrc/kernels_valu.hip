// FP32 wavefront-FMA kernels: the narrow layers (few channels) and the
// FP32 path of any layer.  Every output value is a fixed chain of fmaf in
// tap-major, channel-minor order that does not depend on where a frame sits
// in its buffer, so results are bitwise independent of the buffer split and
// of the other streams in the step.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sc {

namespace {

constexpr int kBlock = 256;
constexpr int kNarrowLdsBytes = 48 * 1024;

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

__device__ inline Row window_row(const Entry& e, int64_t in_start, int64_t Tin, int64_t row, int32_t L,
                                 int64_t soff, int64_t slen, const float* buf, int32_t C) {
  if (row < L) return Row{e.state + soff + (int64_t)e.parity * slen + row * C, 1};
  const int64_t r = row - L;
  if (buf) return Row{buf + (in_start + r) * C, 1};
  return Row{e.in + r, Tin};  // user input, channel-major
}

// New cache of a conv = window rows [Tin, Tin + L), into the other copy.
__device__ inline void cache_item(const LayerArgs& a, int64_t j) {
  const int64_t per_ent = (int64_t)a.L * a.cin;
  const int ei = (int)(j / per_ent);
  const int64_t rem = j % per_ent;
  const int64_t i = rem / a.cin;
  const int ci = (int)(rem % a.cin);
  const Entry e = a.ents[ei];
  const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
  const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
  const Row rw = window_row(e, in_start, Tin, Tin + i, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
  e.state[a.state_off + (int64_t)(1 - e.parity) * a.state_len + i * a.cin + ci] = rw.p[ci * rw.cs];
}

__device__ inline float finish(const LayerArgs& a, const Entry& e, int64_t t, float acc) {
  if (a.post_act == 2) acc = tanhf(acc);
  if ((e.flags & SC_FLAG_WARMUP_MASK) && at_rate(e.pos, a.out_num, a.out_den) + t < a.delay) acc = 0.f;
  return acc;
}

// Per-item conv: one lane per output value (used when the LDS window of the
// narrow kernel would not fit).  Grid-stride over outputs, then cache items.
__global__ void __launch_bounds__(kBlock) conv_item_kernel(LayerArgs a) {
  const int64_t n_items = a.n_out * a.cout;
  const int64_t total = n_items + (int64_t)a.n_ent * a.L * a.cin;
  const float* W = static_cast<const float*>(a.W);
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    if (idx >= n_items) {
      cache_item(a, idx - n_items);
      continue;
    }
    const int co = (int)(idx % a.cout);
    const int64_t n = idx / a.cout;
    const Entry e = a.ents[entry_at(a.fent, n, a.out_num, a.out_den)];
    const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
    const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
    const int64_t t = n - at_rate(e.off, a.out_num, a.out_den);
    float acc = a.B[co];
    for (int kk = 0; kk < a.k; ++kk) {
      const Row rw = window_row(e, in_start, Tin, t * a.stride + (int64_t)a.dil * kk, a.L, a.state_off,
                                a.state_len, a.in_buf, a.cin);
      const float* wp = W + (int64_t)kk * a.cin * a.cout + co;
      for (int ci = 0; ci < a.cin; ++ci) {
        float x = rw.p[ci * rw.cs];
        if (a.pre_act) x = lrelu(x);
        acc = fmaf(wp[(int64_t)ci * a.cout], x, acc);
      }
    }
    if (a.residual) {
      const Row rw = window_row(e, in_start, Tin, t + a.skip_off, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
      acc = acc + rw.p[co * rw.cs];
    }
    acc = finish(a, e, t, acc);
    if (a.out_buf) a.out_buf[n * a.cout + co] = acc;
    else e.out[(int64_t)co * at_rate(e.T, a.out_num, a.out_den) + t] = acc;
  }
}

// LDS-staged narrow conv.  A block owns `a.tile` consecutive output frames of
// the step's packed frame space (possibly of several streams) and a tile of
// output channels.  It stages the activated input rows
// [n0*S - L, (n0 + F)*S) of the packed input once; output frame n, tap k
// reads packed row n*S + d*k - L, which belongs to n's own stream exactly
// when its window row t*S + d*k is >= L -- otherwise the row comes from the
// stream's cache.  Blocks beyond the tiles copy caches.
__global__ void __launch_bounds__(kBlock) conv_narrow_kernel(LayerArgs a, int n_ct, int co_tile, int64_t n_tiles,
                                                             int extra_blocks) {
  extern __shared__ float xs[];
  const int tid = threadIdx.x;
  if ((int64_t)blockIdx.x >= n_tiles) {
    const int64_t total = (int64_t)a.n_ent * a.L * a.cin;
    for (int64_t j = ((int64_t)blockIdx.x - n_tiles) * kBlock + tid; j < total; j += (int64_t)extra_blocks * kBlock)
      cache_item(a, j);
    return;
  }
  const int F = a.tile;
  const int S = a.stride;
  const int ct = (int)(blockIdx.x % n_ct);
  const int64_t n0 = (int64_t)(blockIdx.x / n_ct) * F;
  const int co0 = ct * co_tile;
  const int co_n = min(co_tile, a.cout - co0);
  const int rows = F * S + a.L;
  const int stride = a.cin | 1;          // odd row stride: conflict-free column reads
  const int64_t p0 = n0 * S - a.L;       // packed input row of LDS row 0

  // stage activated input rows
  if (a.in_buf) {
    for (int idx = tid; idx < rows * a.cin; idx += kBlock) {
      const int j = idx / a.cin, ci = idx - j * a.cin;
      const int64_t p = p0 + j;
      float v = 0.f;
      if (p >= 0 && p < a.n_in) v = a.in_buf[p * a.cin + ci];
      xs[j * stride + ci] = a.pre_act ? lrelu(v) : v;
    }
  } else {
    for (int idx = tid; idx < rows * a.cin; idx += kBlock) {
      const int ci = idx / rows, j = idx - ci * rows;   // time fastest: coalesced channel-major reads
      const int64_t p = p0 + j;
      float v = 0.f;
      if (p >= 0 && p < a.n_in) {
        const Entry& e = a.ents[entry_at(a.fent, p, a.in_num, a.in_den)];
        const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
        v = e.in[(int64_t)ci * at_rate(e.T, a.in_num, a.in_den) + (p - in_start)];
      }
      xs[j * stride + ci] = a.pre_act ? lrelu(v) : v;
    }
  }
  __syncthreads();

  const float* W = static_cast<const float*>(a.W);
  const int items = F * co_n;
  for (int it = tid; it < items; it += kBlock) {
    const int i = it / co_n;
    const int co = co0 + (it - i * co_n);
    const int64_t n = n0 + i;
    if (n >= a.n_out) continue;
    const Entry e = a.ents[entry_at(a.fent, n, a.out_num, a.out_den)];
    const int64_t t = n - at_rate(e.off, a.out_num, a.out_den);
    float acc = a.B[co];
    for (int kk = 0; kk < a.k; ++kk) {
      const int64_t w = t * S + (int64_t)a.dil * kk;     // window row
      const float* wp = W + (int64_t)kk * a.cin * a.cout + co;
      if (w >= a.L) {
        const float* x = xs + (i * S + a.dil * kk) * stride;
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], x[ci], acc);
      } else {
        const float* x = e.state + a.state_off + (int64_t)e.parity * a.state_len + w * a.cin;
        for (int ci = 0; ci < a.cin; ++ci) {
          float v = x[ci];
          if (a.pre_act) v = lrelu(v);
          acc = fmaf(wp[(int64_t)ci * a.cout], v, acc);
        }
      }
    }
    if (a.residual) {
      const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
      const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
      const Row rw = window_row(e, in_start, Tin, t + a.skip_off, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
      acc = acc + rw.p[co * rw.cs];
    }
    acc = finish(a, e, t, acc);
    if (a.out_buf) a.out_buf[n * a.cout + co] = acc;
    else e.out[(int64_t)co * at_rate(e.T, a.out_num, a.out_den) + t] = acc;
  }
}

// Transposed conv, kernel 2r: output frame q*r + phi of a buffer is
//   W[phi + r] . a[q-1] + W[phi] . a[q]   (+ bias),
// accumulated in that order.  Columns [0, n_in) are the input frames q of all
// streams; columns n_in + e hold, for stream e, only the first half of
// q = T: that is the FP32 overlap carry that column q = 0 of the next buffer
// starts from, so the chain of fmaf is the same for every frame.
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
    const int ei = c < a.n_in ? entry_at(a.fent, c, a.in_num, a.in_den) : (int)(c - a.n_in);
    const Entry e = a.ents[ei];
    const int64_t in_start = at_rate(e.off, a.in_num, a.in_den);
    const int64_t Tin = at_rate(e.T, a.in_num, a.in_den);
    const int64_t q = c < a.n_in ? c - in_start : Tin;
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
      if (a.out_buf) a.out_buf[(in_start * r + t) * a.cout + co] = v;
      else e.out[(int64_t)co * (Tin * r) + t] = v;
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
      const Entry e = a.ents[entry_at(a.fent, n, a.out_num, a.out_den)];
      const int64_t start = at_rate(e.off, a.out_num, a.out_den);
      const int64_t Tn = at_rate(e.T, a.out_num, a.out_den);
      const int64_t t = n - start;
      const Row r0 = window_row(e, start, Tn, t, a.A0, a.state_off, a.state_len, a.in_buf, C);
      const Row r1 = window_row(e, start, Tn, t, a.A1, a.state_off2, a.state_len2, a.in_buf2, C);
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
      const Row rw = window_row(e, start, Tn, Tn + i, A, soff, slen, second ? a.in_buf2 : a.in_buf, C);
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
      const Entry e = a.ents[entry_at(a.fent, n, a.in_num, a.in_den)];
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

int32_t narrow_conv_tile(int cin, int cout, int k, int dil, int stride, int L, int64_t n_out_hint) {
  (void)k;
  (void)dil;
  const int stride_f = cin | 1;
  int F = 256;
  while (F > 16 && (int64_t)(F * stride + L) * stride_f * 4 > kNarrowLdsBytes) F /= 2;
  if ((int64_t)(F * stride + L) * stride_f * 4 > kNarrowLdsBytes) return 0;
  // enough blocks to fill the chip when outputs are many channels wide
  const int co_tile = cout < kBlock ? cout : kBlock;
  const int n_ct = (cout + co_tile - 1) / co_tile;
  while (F > 16 && n_out_hint > 0 && ((n_out_hint + F - 1) / F) * n_ct < 1024 && F * co_tile > 8 * kBlock) F /= 2;
  return F;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_conv_valu(const LayerArgs& a, hipStream_t s) {
  if (a.tile <= 0) {
    const int64_t items = a.n_out * a.cout + (int64_t)a.n_ent * a.L * a.cin;
    hipLaunchKernelGGL(conv_item_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
  const int co_tile = a.cout < kBlock ? a.cout : kBlock;
  const int n_ct = (a.cout + co_tile - 1) / co_tile;
  const int64_t n_tiles = (a.n_out + a.tile - 1) / a.tile * n_ct;
  const int64_t cache_items = (int64_t)a.n_ent * a.L * a.cin;
  const int extra = (int)std::min<int64_t>((cache_items + kBlock - 1) / kBlock, 1024);
  const size_t lds = (size_t)(a.tile * a.stride + a.L) * (a.cin | 1) * sizeof(float);
  if (n_tiles + extra == 0) return hipSuccess;
  hipLaunchKernelGGL(conv_narrow_kernel, dim3((unsigned)(n_tiles + extra)), dim3(kBlock), lds, s, a, n_ct, co_tile,
                     n_tiles, extra);
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
