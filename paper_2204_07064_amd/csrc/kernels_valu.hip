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
constexpr int kChansC = 16;         // channel-parallel conv: cin and k bounds of the
constexpr int kChansK = 4;          // register-resident weights

typedef float f4v __attribute__((ext_vector_type(4)));

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

__device__ inline Row window_row(const Entry& e, int32_t in_start, int32_t Tin, int32_t row, int32_t L,
                                 int64_t soff, int64_t slen, const float* buf, int32_t C) {
  if (row < L) return Row{e.state + soff + (int64_t)e.parity * slen + (int64_t)row * C, 1};
  const int32_t r = row - L;
  if (buf) return Row{buf + ((int64_t)in_start + r) * C, 1};
  return Row{e.in + r, Tin};  // user input, channel-major
}

// New cache of a conv = window rows [Tin, Tin + L), into the other copy.
// Item j of the step's cache items: entry j / (L*cin), row, channel.
__device__ inline void cache_item(const LayerArgs& a, const FastDiv& fd_per_ent, int32_t j) {
  const int32_t per_ent = a.L * a.cin;
  const int ei = (int)fdiv(fd_per_ent, (uint32_t)j);
  const int32_t rem = j - ei * per_ent;
  const int32_t i = (int32_t)fdiv(a.fd_cin, (uint32_t)rem);
  const int ci = rem - i * a.cin;
  const Entry e = load_entry(a.ents + ei);
  const int32_t in_start = in_frames(a, e.off);
  const int32_t Tin = in_frames(a, e.T);
  const Row rw = window_row(e, in_start, Tin, Tin + i, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
  gstore<float>(e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len + (int64_t)i * a.cin + ci,
                gload<float>(rw.p + ci * rw.cs));
}

__device__ inline float finish(const LayerArgs& a, const Entry& e, int32_t t, float acc) {
  if (a.post_act == 2) acc = tanhf(acc);
  if (masked(a, e, t)) acc = 0.f;
  return acc;
}

// Per-item conv: one lane per output value (used when the LDS window of the
// narrow kernel would not fit).  Grid-stride over outputs, then cache items.
__global__ void __launch_bounds__(kBlock) conv_item_kernel(LayerArgs a, FastDiv fd_per_ent) {
  const int32_t n_items = (int32_t)step_out(a) * a.cout;
  const int32_t total = n_items + step_ents(a) * a.L * a.cin;
  const float* W = static_cast<const float*>(a.W);
  for (int32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < total; idx += gridDim.x * kBlock) {
    if (idx >= n_items) {
      cache_item(a, fd_per_ent, idx - n_items);
      continue;
    }
    const int32_t n = (int32_t)fdiv(a.fd_cout, (uint32_t)idx);
    const int co = idx - n * a.cout;
    const Entry e = load_entry(a.ents + entry_of_out(a, n));
    const int32_t in_start = in_frames(a, e.off);
    const int32_t Tin = in_frames(a, e.T);
    const int32_t t = n - out_frames(a, e.off);
    float acc = a.B[co];
    for (int kk = 0; kk < a.k; ++kk) {
      const Row rw = window_row(e, in_start, Tin, t * a.stride + a.dil * kk, a.L, a.state_off, a.state_len,
                                a.in_buf, a.cin);
      const float* wp = W + (int64_t)kk * a.cin * a.cout + co;
      for (int ci = 0; ci < a.cin; ++ci) {
        float x = gload<float>(rw.p + ci * rw.cs);
        if (a.pre_act) x = lrelu(x);
        acc = fmaf(wp[(int64_t)ci * a.cout], x, acc);
      }
    }
    if (a.residual) {
      const Row rw = window_row(e, in_start, Tin, t + a.skip_off, a.L, a.state_off, a.state_len, a.in_buf, a.cin);
      acc = acc + gload<float>(rw.p + co * rw.cs);
    }
    acc = finish(a, e, t, acc);
    if (a.out_buf) {
      a.out_buf[(int64_t)n * a.cout + co] = acc;
      if (a.out_twin) store_twin1(a.out_twin, (int64_t)n * a.cout + co, a.twin_prec, a.twin_pre, a.twin_qs, acc);
    } else {
      gstore<float>(e.out + (int64_t)co * out_frames(a, e.T) + t, acc);
    }
  }
}

// ---- LDS-staged narrow convs ---------------------------------------------------
// A block owns F consecutive output frames of the step's packed frame space
// (possibly of several streams).  It stages the activated input rows
// [n0*S - L, (n0 + F)*S) of the packed input once; output frame n, tap k
// reads packed row n*S + d*k - L, which belongs to n's own stream exactly when
// its window row t*S + d*k is >= L -- otherwise the row comes from the
// stream's cache.  Per-frame stream data is resolved once per block into LDS.
// Blocks beyond the tiles copy caches.
struct FrameInfo {
  const float* cache;   // current cache copy of the frame's stream
  float* out;           // user output: &out[t] of the stream (channel stride `tout`)
  int32_t t;            // local output frame
  int32_t tout;         // output frames of the stream in this step
  int32_t masked;       // warm-up mask applies
  int32_t ei;
};

constexpr int kStageUnroll = 8;
// Streams of a tile whose cache rows are staged in LDS (a tile spans
// consecutive streams; beyond this many, later ones read their cache directly).
constexpr int kCacheSlots = 8;

// Stages the activated cache rows [0, L) of the tile's first kCacheSlots
// streams e_first, e_first + 1, ... into cs (row stride ld).
__device__ inline void stage_cache(const LayerArgs& a, float* cs, int e_first, int e_last, int ld) {
  const int slots = min(e_last - e_first + 1, kCacheSlots);
  const int per = a.L * a.cin;
  for (int idx = threadIdx.x; idx < slots * per; idx += kBlock) {
    const int s = (int)fdiv(a.fd_per_ent_narrow, (uint32_t)idx);
    const int rem = idx - s * per;
    const int w = (int)fdiv(a.fd_cin, (uint32_t)rem);
    const int ci = rem - w * a.cin;
    const Entry e = load_entry(a.ents + e_first + s);
    const float v = gload<float>(e.state + a.state_off + (int64_t)e.parity * a.state_len + rem);
    cs[(s * a.L + w) * ld + ci] = a.pre_act ? lrelu(v) : v;
  }
}

// Stages rows [p0, p0 + rows) x cin (activated) into xs with row stride `ld`.
__device__ inline void stage_rows(const LayerArgs& a, float* xs, int64_t p0, int rows, int ld) {
  const int tid = threadIdx.x;
  if (a.in_buf && (a.cin & 3) == 0) {
    // the rows are one contiguous range of the packed buffer: float4 copies,
    // several loads in flight per thread before the LDS writes
    const int64_t base = p0 * a.cin;
    const int64_t lim = step_in(a) * a.cin;
    const int total4 = rows * a.cin / 4;
    for (int v0 = 0; v0 < total4; v0 += kBlock * kStageUnroll) {
      f4v buf[kStageUnroll];
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) {
        const int v = v0 + u * kBlock + tid;
        const int64_t g = base + (int64_t)v * 4;
        buf[u] = (v < total4 && g >= 0 && g < lim) ? *reinterpret_cast<const f4v*>(a.in_buf + g) : f4v{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) {
        const int v = v0 + u * kBlock + tid;
        if (v >= total4) break;
        const int e0 = v * 4;
        const int j = (int)fdiv(a.fd_cin, (uint32_t)e0), ci = e0 - j * a.cin;
        float* d = xs + j * ld + ci;
        const f4v x = buf[u];
        d[0] = a.pre_act ? lrelu(x.x) : x.x;
        d[1] = a.pre_act ? lrelu(x.y) : x.y;
        d[2] = a.pre_act ? lrelu(x.z) : x.z;
        d[3] = a.pre_act ? lrelu(x.w) : x.w;
      }
    }
    return;
  }
  const int total = rows * a.cin;
  for (int v0 = 0; v0 < total; v0 += kBlock * kStageUnroll) {
    float buf[kStageUnroll];
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int idx = v0 + u * kBlock + tid;
      float v = 0.f;
      if (idx < total) {
        const int j = (int)fdiv(a.fd_cin, (uint32_t)idx), ci = idx - j * a.cin;
        const int64_t p = p0 + j;
        if (p >= 0 && p < step_in(a)) v = a.in_buf[p * a.cin + ci];
      }
      buf[u] = v;
    }
#pragma unroll
    for (int u = 0; u < kStageUnroll; ++u) {
      const int idx = v0 + u * kBlock + tid;
      if (idx >= total) break;
      const int j = (int)fdiv(a.fd_cin, (uint32_t)idx), ci = idx - j * a.cin;
      xs[j * ld + ci] = a.pre_act ? lrelu(buf[u]) : buf[u];
    }
  }
}

__device__ inline void frame_infos(const LayerArgs& a, FrameInfo* fi, int32_t n0, int F) {
  for (int i = threadIdx.x; i < F; i += kBlock) {
    FrameInfo f;
    f.cache = nullptr;
    f.out = nullptr;
    f.t = 0;
    f.tout = 0;
    f.masked = 0;
    f.ei = -1;
    const int32_t n = n0 + i;
    if (n < step_out(a)) {
      const int ei = entry_of_out(a, n);
      const Entry e = load_entry(a.ents + ei);
      const int32_t t = n - out_frames(a, e.off);
      f.ei = ei;
      f.t = t;
      f.tout = out_frames(a, e.T);
      f.cache = e.state + a.state_off + (int64_t)e.parity * a.state_len;
      f.out = e.out + t;
      f.masked = masked(a, e, t);
    }
    fi[i] = f;
  }
}

// Raw (not activated) skip value of window row t + skip_off, channel co.
__device__ inline float skip_value(const LayerArgs& a, const FrameInfo& f, int co) {
  const int32_t row = f.t + a.skip_off;
  if (row < a.L) return gload<float>(f.cache + (int64_t)row * a.cin + co);
  const int32_t off = ((cptr<Entry>)a.ents)[f.ei].off;
  return gload<float>(a.in_buf + ((int64_t)in_frames(a, off) + row - a.L) * a.cin + co);
}

// Frame-parallel variant (few output channels): one lane per output frame,
// looping over the output channels; weights staged in LDS.
__global__ void __launch_bounds__(kBlock) conv_frames_kernel(LayerArgs a, int32_t n_tiles, int extra_blocks,
                                                             FastDiv fd_per_ent) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  if ((int32_t)blockIdx.x >= n_tiles) {
    const int32_t total = step_ents(a) * a.L * a.cin;
    for (int32_t j = ((int32_t)blockIdx.x - n_tiles) * kBlock + tid; j < total; j += extra_blocks * kBlock)
      cache_item(a, fd_per_ent, j);
    return;
  }
  const int F = a.tile, S = a.stride, ld = a.cin | 1;
  const int rows = F * S + a.L;
  const int nw = a.k * a.cin * a.cout;
  float* ws = smem;                                   // [k][cin][cout]
  FrameInfo* fi = reinterpret_cast<FrameInfo*>(smem + ((nw + 3) & ~3));
  float* xs = reinterpret_cast<float*>(fi + F);
  float* cs = xs + rows * ld;                          // cache rows of the tile's streams
  const int32_t n0 = (int32_t)blockIdx.x * F;
  if (n0 >= step_out(a)) return;                       // grid sized for the largest step
  const float* W = static_cast<const float*>(a.W);
  const int e_first = entry_of_out(a, n0);
  const int e_last = entry_of_out(a, min((int32_t)(n0 + F), (int32_t)step_out(a)) - 1);
  for (int i = tid; i < nw; i += kBlock) ws[i] = W[i];
  frame_infos(a, fi, n0, F);
  stage_rows(a, xs, (int64_t)n0 * S - a.L, rows, ld);
  stage_cache(a, cs, e_first, e_last, ld);
  __syncthreads();
  if (a.out_buf && (a.cout & 3) == 0) {
    // one lane per (frame, 4 output channels): each output summed as below,
    // one 16-byte store (and one twin store) per lane
    const int c4 = a.cout >> 2;
    for (int idx = tid; idx < F * c4; idx += kBlock) {
      const int i = idx / c4;
      const int co = (idx - i * c4) * 4;
      const FrameInfo f = fi[i];
      if (f.ei < 0) continue;
      float acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = a.B[co + j];
      for (int kk = 0; kk < a.k; ++kk) {
        const int w = f.t * S + a.dil * kk;       // window row
        const float* wp = ws + kk * a.cin * a.cout + co;
        // the row in LDS (staged input or cache rows), else the stream's cache in memory
        const bool in_lds = w >= a.L || f.ei - e_first < kCacheSlots;
        const float* x = w >= a.L ? xs + (i * S + a.dil * kk) * ld : cs + ((f.ei - e_first) * a.L + w) * ld;
        if (in_lds) {
          for (int ci = 0; ci < a.cin; ++ci) {
            const float xv = x[ci];
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = fmaf(wp[ci * a.cout + j], xv, acc[j]);
          }
        } else {
          const float* xg = f.cache + (int64_t)w * a.cin;
          for (int ci = 0; ci < a.cin; ++ci) {
            float v = gload<float>(xg + ci);
            if (a.pre_act) v = lrelu(v);
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] = fmaf(wp[ci * a.cout + j], v, acc[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (a.residual) acc[j] = acc[j] + skip_value(a, f, co + j);
        if (a.post_act == 2) acc[j] = tanhf(acc[j]);
        if (f.masked) acc[j] = 0.f;
      }
      const int64_t o = (int64_t)(n0 + i) * a.cout + co;
      *reinterpret_cast<f4v*>(a.out_buf + o) = f4v{acc[0], acc[1], acc[2], acc[3]};
      if (a.out_twin) store_twin4v(a.out_twin, o, a.twin_prec, a.twin_pre, a.twin_qs, acc[0], acc[1], acc[2], acc[3]);
    }
    return;
  }
  // one lane per (frame, output channel): consecutive lanes write consecutive
  // channels of a frame
  for (int idx = tid; idx < F * a.cout; idx += kBlock) {
    const int i = (int)fdiv(a.fd_cout, (uint32_t)idx);
    const int co = idx - i * a.cout;
    const FrameInfo f = fi[i];
    if (f.ei < 0) continue;
    float acc = a.B[co];
    for (int kk = 0; kk < a.k; ++kk) {
      const int w = f.t * S + a.dil * kk;       // window row
      const float* wp = ws + kk * a.cin * a.cout + co;
      if (w >= a.L) {
        const float* x = xs + (i * S + a.dil * kk) * ld;
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[ci * a.cout], x[ci], acc);
      } else if (f.ei - e_first < kCacheSlots) {
        const float* x = cs + ((f.ei - e_first) * a.L + w) * ld;
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[ci * a.cout], x[ci], acc);
      } else {
        const float* x = f.cache + (int64_t)w * a.cin;
        for (int ci = 0; ci < a.cin; ++ci) {
          float v = gload<float>(x + ci);
          if (a.pre_act) v = lrelu(v);
          acc = fmaf(wp[ci * a.cout], v, acc);
        }
      }
    }
    if (a.residual) acc = acc + skip_value(a, f, co);
    if (a.post_act == 2) acc = tanhf(acc);
    if (f.masked) acc = 0.f;
    if (a.out_buf) {
      a.out_buf[(n0 + i) * a.cout + co] = acc;
      if (a.out_twin) store_twin1(a.out_twin, (n0 + i) * a.cout + co, a.twin_prec, a.twin_pre, a.twin_qs, acc);
    } else {
      gstore<float>(f.out + (int64_t)co * f.tout, acc);
    }
  }
}

// Channel-parallel variant (many output channels, short reductions): a block
// owns a tile of F frames and kChansCo output channels; the tile's weights are
// staged in LDS with vector loads, then each lane keeps the weights of its
// channel in registers (cin <= CMAX, k <= KMAX) and walks half of the frames;
// input rows are LDS broadcasts.
constexpr int kChansCo = 128;

template <int CMAX, int KMAX>
__global__ void __launch_bounds__(kBlock) conv_chans_kernel(LayerArgs a, int32_t n_tiles, int extra_blocks,
                                                            FastDiv fd_per_ent, int n_ct) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  if ((int32_t)blockIdx.x >= n_tiles) {
    const int32_t total = step_ents(a) * a.L * a.cin;
    for (int32_t j = ((int32_t)blockIdx.x - n_tiles) * kBlock + tid; j < total; j += extra_blocks * kBlock)
      cache_item(a, fd_per_ent, j);
    return;
  }
  const int F = a.tile, S = a.stride, ld = a.cin | 1;
  const int rows = F * S + a.L;
  const int kin = a.k * a.cin;
  const int ct = (int)((uint32_t)blockIdx.x % (uint32_t)n_ct);
  const int32_t n0 = (int32_t)((uint32_t)blockIdx.x / (uint32_t)n_ct) * F;
  if (n0 >= step_out(a)) return;                       // grid sized for the largest step
  const int co0 = ct * kChansCo;
  float* wsm = smem;                                   // [kin][kChansCo]
  FrameInfo* fi = reinterpret_cast<FrameInfo*>(wsm + kin * kChansCo);
  float* xs = reinterpret_cast<float*>(fi + F);
  float* cs = xs + rows * ld;                          // cache rows of the tile's streams
  const int e_first = entry_of_out(a, n0);
  const int e_last = entry_of_out(a, min((int32_t)(n0 + F), (int32_t)step_out(a)) - 1);
  {
    // weight tile: rows q of W[q][cout] (q = tap * cin + ci), columns co0..co0+127
    const float* W = static_cast<const float*>(a.W);
    const int n4 = kin * (kChansCo / 4);
    for (int v = tid; v < n4; v += kBlock) {
      const int q = v >> 5, c4 = (v & 31) * 4;        // kChansCo / 4 == 32 vectors per row
      f4v w = {0.f, 0.f, 0.f, 0.f};
      if (co0 + c4 < a.cout) w = *reinterpret_cast<const f4v*>(W + (int64_t)q * a.cout + co0 + c4);
      *reinterpret_cast<f4v*>(wsm + q * kChansCo + c4) = w;
    }
  }
  frame_infos(a, fi, n0, F);
  stage_rows(a, xs, (int64_t)n0 * S - a.L, rows, ld);
  stage_cache(a, cs, e_first, e_last, ld);
  __syncthreads();
  const int cl = tid & (kChansCo - 1);
  const int co = co0 + cl;
  if (co >= a.cout) return;
  float wr[KMAX][CMAX];
#pragma unroll
  for (int kk = 0; kk < KMAX; ++kk)
#pragma unroll
    for (int ci = 0; ci < CMAX; ++ci)
      wr[kk][ci] = (kk < a.k && ci < a.cin) ? wsm[(kk * a.cin + ci) * kChansCo + cl] : 0.f;
  const float bias = a.B[co];
  for (int i = tid >> 7; i < F; i += kBlock / kChansCo) {
    const FrameInfo f = fi[i];
    if (f.ei < 0) break;
    float acc = bias;
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
      if (kk >= a.k) break;
      const int w = f.t * S + a.dil * kk;
      if (w >= a.L) {
        const float* x = xs + (i * S + a.dil * kk) * ld;
#pragma unroll
        for (int ci = 0; ci < CMAX; ++ci)
          if (ci < a.cin) acc = fmaf(wr[kk][ci], x[ci], acc);
      } else if (f.ei - e_first < kCacheSlots) {
        const float* x = cs + ((f.ei - e_first) * a.L + w) * ld;
#pragma unroll
        for (int ci = 0; ci < CMAX; ++ci)
          if (ci < a.cin) acc = fmaf(wr[kk][ci], x[ci], acc);
      } else {
        const float* x = f.cache + (int64_t)w * a.cin;
#pragma unroll
        for (int ci = 0; ci < CMAX; ++ci) {
          if (ci < a.cin) {
            float v = gload<float>(x + ci);
            if (a.pre_act) v = lrelu(v);
            acc = fmaf(wr[kk][ci], v, acc);
          }
        }
      }
    }
    if (a.residual) acc = acc + skip_value(a, f, co);
    if (a.post_act == 2) acc = tanhf(acc);
    if (f.masked) acc = 0.f;
    if (a.out_buf) {
      a.out_buf[(int64_t)(n0 + i) * a.cout + co] = acc;
      if (a.out_twin) store_twin1(a.out_twin, (int64_t)(n0 + i) * a.cout + co, a.twin_prec, a.twin_pre, a.twin_qs, acc);
    } else {
      gstore<float>(f.out + (int64_t)co * f.tout, acc);
    }
  }
}

// One-output-channel conv with compile-time input width (the decoder's output
// conv): one lane per frame, taps and channels fully unrolled over 16-byte LDS
// reads (rows padded to CIN + 4 floats), weights broadcast from LDS.
template <int CIN, int KMAX>
__global__ void __launch_bounds__(kBlock) conv_out1_kernel(LayerArgs a, int32_t n_tiles, int extra_blocks,
                                                           FastDiv fd_per_ent) {
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  if ((int32_t)blockIdx.x >= n_tiles) {
    const int32_t total = step_ents(a) * a.L * a.cin;
    for (int32_t j = ((int32_t)blockIdx.x - n_tiles) * kBlock + tid; j < total; j += extra_blocks * kBlock)
      cache_item(a, fd_per_ent, j);
    return;
  }
  constexpr int LD = CIN + 4;
  const int F = a.tile;
  const int rows = F + a.L;
  float* ws = smem;                                    // [KMAX][CIN] (taps >= k are zero)
  FrameInfo* fi = reinterpret_cast<FrameInfo*>(ws + KMAX * CIN);
  float* xs = reinterpret_cast<float*>(fi + F);        // [rows][LD]
  float* cs = xs + rows * LD;                          // [kCacheSlots][L][LD]
  const int32_t n0 = (int32_t)blockIdx.x * F;
  if (n0 >= step_out(a)) return;                       // grid sized for the largest step
  const int e_first = entry_of_out(a, n0);
  const int e_last = entry_of_out(a, min((int32_t)(n0 + F), (int32_t)step_out(a)) - 1);
  const float* W = static_cast<const float*>(a.W);
  for (int q = tid; q < KMAX * CIN; q += kBlock) ws[q] = q < a.k * CIN ? W[q] : 0.f;
  frame_infos(a, fi, n0, F);
  stage_rows(a, xs, (int64_t)n0 - a.L, rows, LD);
  stage_cache(a, cs, e_first, e_last, LD);
  __syncthreads();
  for (int i = tid; i < F; i += kBlock) {
    const FrameInfo f = fi[i];
    if (f.ei < 0) break;
    float acc = a.B[0];
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
      if (kk < a.k) {
        const int w = f.t + a.dil * kk;
        // the row in LDS (staged input or cache rows), else the stream's cache in memory
        const bool in_lds = w >= a.L || f.ei - e_first < kCacheSlots;
        const float* x = w >= a.L ? xs + (i + a.dil * kk) * LD : cs + ((f.ei - e_first) * a.L + w) * LD;
        if (in_lds) {
#pragma unroll
          for (int c4 = 0; c4 < CIN; c4 += 4) {
            const f4v xv = *reinterpret_cast<const f4v*>(x + c4);
            const f4v wv = *reinterpret_cast<const f4v*>(ws + kk * CIN + c4);
            acc = fmaf(wv.x, xv.x, acc);
            acc = fmaf(wv.y, xv.y, acc);
            acc = fmaf(wv.z, xv.z, acc);
            acc = fmaf(wv.w, xv.w, acc);
          }
        } else {
          const float* xg = f.cache + (int64_t)w * CIN;
          for (int ci = 0; ci < CIN; ++ci) {
            float v = gload<float>(xg + ci);
            if (a.pre_act) v = lrelu(v);
            acc = fmaf(ws[kk * CIN + ci], v, acc);
          }
        }
      }
    }
    if (a.post_act == 2) acc = tanhf(acc);
    if (f.masked) acc = 0.f;
    if (a.out_buf) {
      a.out_buf[n0 + i] = acc;
      if (a.out_twin) store_twin1(a.out_twin, n0 + i, a.twin_prec, a.twin_pre, a.twin_qs, acc);
    } else {
      gstore<float>(f.out, acc);
    }
  }
}

// Channel-major user input [C][T] of every stream -> packed channels-last
// [frame][C] for the step.
__global__ void __launch_bounds__(kBlock) pack_input_kernel(const Entry* ents, const int32_t* fent, FastDiv fd_gran,
                                                           const int32_t* hdr, int32_t C, float* out, void* twin,
                                                           int32_t twin_prec, int32_t twin_pre, float twin_qs) {
  const int32_t n_frames = ((cptr<int32_t>)hdr)[1];
  const int32_t total = n_frames * C;
  for (int32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < total; idx += gridDim.x * kBlock) {
    const int c = idx / n_frames;   // frame fastest: coalesced reads of each channel row
    const int32_t f = idx - c * n_frames;
    const Entry e = load_entry(ents + fent[fdiv(fd_gran, (uint32_t)f)]);
    const float v = gload<float>(e.in + (int64_t)c * e.T + (f - e.off));
    out[(int64_t)f * C + c] = v;
    if (twin) store_twin1(twin, (int64_t)f * C + c, twin_prec, twin_pre, twin_qs, v);
  }
}

// Transposed conv, kernel 2r: output frame q*r + phi of a buffer is
//   W[phi + r] . a[q-1] + W[phi] . a[q]   (+ bias),
// accumulated in that order.  Columns [0, n_in) are the input frames q of all
// streams; columns n_in + e hold, for stream e, only the first half of
// q = T: that is the FP32 overlap carry that column q = 0 of the next buffer
// starts from, so the chain of fmaf is the same for every frame.
// Weights packed [h][phi][cin][cout], h = 0 -> tap phi + r, h = 1 -> tap phi.
__global__ void __launch_bounds__(kBlock) convt_valu_kernel(LayerArgs a, FastDiv fd_r) {
  const int r = a.stride;
  const int32_t n_cols = (int32_t)step_in(a) + step_ents(a);
  const int32_t total = n_cols * r * a.cout;
  const float* W = static_cast<const float*>(a.W);
  for (int32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < total; idx += gridDim.x * kBlock) {
    const int32_t rest = (int32_t)fdiv(a.fd_cout, (uint32_t)idx);
    const int co = idx - rest * a.cout;
    const int32_t c = (int32_t)fdiv(fd_r, (uint32_t)rest);
    const int phi = rest - c * r;
    const int ei = c < step_in(a) ? entry_of_in(a, c) : c - (int32_t)step_in(a);
    const Entry e = load_entry(a.ents + ei);
    const int32_t in_start = in_frames(a, e.off);
    const int32_t Tin = in_frames(a, e.T);
    const int32_t q = c < step_in(a) ? c - in_start : Tin;
    const float* carry_in = e.state + a.state_off + (int64_t)e.parity * a.state_len;
    float acc = (q == 0) ? gload<float>(carry_in + phi * a.cout + co) : 0.f;
    for (int h = 0; h < 2; ++h) {
      const int32_t row = q - 1 + h;
      if (row < 0 || row >= Tin) continue;
      const float* x = a.in_buf + ((int64_t)in_start + row) * a.cin;
      const float* wp = W + ((int64_t)(h * r + phi) * a.cin) * a.cout + co;
      if (a.pre_act) {
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], lrelu(x[ci]), acc);
      } else {
        for (int ci = 0; ci < a.cin; ++ci) acc = fmaf(wp[(int64_t)ci * a.cout], x[ci], acc);
      }
    }
    if (q < Tin) {
      float v = acc + a.B[co];
      const int32_t t = q * r + phi;
      if (masked(a, e, t)) v = 0.f;
      if (a.out_buf) {
        const int64_t o = ((int64_t)in_start * r + t) * a.cout + co;
        a.out_buf[o] = v;
        if (a.out_twin) store_twin1(a.out_twin, o, a.twin_prec, a.twin_pre, a.twin_qs, v);
      } else {
        gstore<float>(e.out + (int64_t)co * (Tin * r) + t, v);
      }
    } else {
      gstore<float>(e.state + a.state_off + (int64_t)(1 - e.parity) * a.state_len + phi * a.cout + co, acc);
    }
  }
}

// Sum of two branches, branch j delayed by A_j frames through a delay line
// (Eq. 3).  Window of branch j: [line_j (A_j frames) | new frames].
__global__ void __launch_bounds__(kBlock) delay_add_kernel(LayerArgs a, FastDiv fd_per_ent) {
  const int C = a.cout;
  const int32_t n_items = (int32_t)step_out(a) * C;
  const int32_t per_ent = (a.A0 + a.A1) * C;
  const int32_t total = n_items + step_ents(a) * per_ent;
  for (int32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < total; idx += gridDim.x * kBlock) {
    if (idx < n_items) {
      const int32_t n = (int32_t)fdiv(a.fd_cout, (uint32_t)idx);
      const int c = idx - n * C;
      const Entry e = load_entry(a.ents + entry_of_out(a, n));
      const int32_t start = out_frames(a, e.off);
      const int32_t Tn = out_frames(a, e.T);
      const int32_t t = n - start;
      const Row r0 = window_row(e, start, Tn, t, a.A0, a.state_off, a.state_len, a.in_buf, C);
      const Row r1 = window_row(e, start, Tn, t, a.A1, a.state_off2, a.state_len2, a.in_buf2, C);
      float v = gload<float>(r0.p + c * r0.cs) + gload<float>(r1.p + c * r1.cs);
      if (masked(a, e, t)) v = 0.f;
      if (a.out_buf) {
        a.out_buf[(int64_t)n * C + c] = v;
        if (a.out_twin) store_twin1(a.out_twin, (int64_t)n * C + c, a.twin_prec, a.twin_pre, a.twin_qs, v);
      } else {
        gstore<float>(e.out + (int64_t)c * Tn + t, v);
      }
    } else {
      const int32_t j = idx - n_items;
      const int ei = (int)fdiv(fd_per_ent, (uint32_t)j);
      int32_t rem = j - ei * per_ent;
      const Entry e = load_entry(a.ents + ei);
      const int32_t start = out_frames(a, e.off);
      const int32_t Tn = out_frames(a, e.T);
      const bool second = rem >= a.A0 * C;
      if (second) rem -= a.A0 * C;
      const int32_t i = (int32_t)fdiv(a.fd_cout, (uint32_t)rem);
      const int c = rem - i * C;
      const int32_t A = second ? a.A1 : a.A0;
      const int64_t soff = second ? a.state_off2 : a.state_off;
      const int64_t slen = second ? a.state_len2 : a.state_len;
      const Row rw = window_row(e, start, Tn, Tn + i, A, soff, slen, second ? a.in_buf2 : a.in_buf, C);
      gstore<float>(e.state + soff + (int64_t)(1 - e.parity) * slen + (int64_t)i * C + c, gload<float>(rw.p + c * rw.cs));
    }
  }
}

__global__ void __launch_bounds__(kBlock) amax_kernel(LayerArgs a, float* amax) {
  __shared__ float red[kBlock];
  float m = 0.f;
  const int64_t total = step_in(a) * a.cin;
  for (int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * kBlock) {
    float v = a.in_buf[idx];
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

// 16-byte pieces, then the last bytes % 16 bytes one by one (16-byte aligned ends)
__global__ void __launch_bounds__(kBlock) upload_kernel(const unsigned char* __restrict__ src,
                                                       unsigned char* __restrict__ dst, int64_t bytes) {
  const int64_t n = bytes / 16;
  const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t i = first; i < n; i += (int64_t)gridDim.x * kBlock)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  if (first < bytes - n * 16) dst[n * 16 + first] = src[n * 16 + first];
}

}  // namespace

// Narrow-conv kernel choice: 1 = channel-parallel, 2 = frame-parallel,
// 3 = one-output-channel with compile-time width, 0 = per item.
static int narrow_kind(int cin, int cout, int k, int stride, int residual) {
  if (cout == 1 && stride == 1 && !residual && k <= 8 && (cin == 16 || cin == 32 || cin == 48)) return 3;
  if (cout >= 32 && cout % 4 == 0 && cin <= kChansC && k <= kChansK) return 1;
  if (cout <= 16 && k * cin * cout <= 4096) return 2;
  return 0;
}

static size_t narrow_lds(int kind, int F, int cin, int cout, int k, int stride, int L) {
  if (kind == 3) {
    const int ld = cin + 4;
    return (size_t)(8 * cin + (F + L) * ld + kCacheSlots * L * ld) * sizeof(float) + (size_t)F * sizeof(FrameInfo);
  }
  size_t b = (size_t)(F * stride + L) * (cin | 1) * sizeof(float) + (size_t)F * sizeof(FrameInfo);
  b += (size_t)kCacheSlots * L * (cin | 1) * sizeof(float);
  if (kind == 2) b += (size_t)((k * cin * cout + 3) & ~3) * sizeof(float);
  if (kind == 1) b += (size_t)k * cin * kChansCo * sizeof(float);
  return b;
}

int32_t narrow_conv_tile(int cin, int cout, int k, int dil, int stride, int L, int64_t n_out_hint) {
  (void)dil;
  const int kind = narrow_kind(cin, cout, k, stride, 0);
  if (kind == 0) return 0;
  int F = 256;
  while (F > 8 && narrow_lds(kind, F, cin, cout, k, stride, L) > kNarrowLdsBytes) F /= 2;
  if (narrow_lds(kind, F, cin, cout, k, stride, L) > kNarrowLdsBytes) return 0;
  if (kind == 1) {
    // channel-parallel: two frames per lane pass; keep tiles short enough to
    // give every CU a few blocks
    const int n_ct = (cout + kChansCo - 1) / kChansCo;
    while (F > 8 && n_out_hint > 0 && (n_out_hint + F - 1) / F * n_ct < 1024) F /= 2;
  }
  return F;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_upload(const void* src, void* dst, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(upload_kernel, dim3(grid_for((int64_t)(bytes + 15) / 16)), dim3(kBlock), 0, s,
                     static_cast<const unsigned char*>(src), static_cast<unsigned char*>(dst), (int64_t)bytes);
  return hipGetLastError();
}

hipError_t launch_conv_valu(const LayerArgs& a, hipStream_t s) {
  const int kind = a.tile > 0 ? narrow_kind(a.cin, a.cout, a.k, a.stride, a.residual) : 0;
  const FastDiv fpe = make_fastdiv((uint32_t)std::max(a.L * a.cin, 1));
  if (kind == 0) {
    const int64_t items = a.n_out * a.cout + (int64_t)a.n_ent * a.L * a.cin;
    hipLaunchKernelGGL(conv_item_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a, fpe);
    return hipGetLastError();
  }
  const int n_ct = kind == 1 ? (a.cout + kChansCo - 1) / kChansCo : 1;
  const int64_t n_tiles = (a.n_out + a.tile - 1) / a.tile * n_ct;
  const int64_t cache_items = (int64_t)a.n_ent * a.L * a.cin;
  const int extra = (int)std::min<int64_t>((cache_items + kBlock - 1) / kBlock, 1024);
  const size_t lds = narrow_lds(kind, a.tile, a.cin, a.cout, a.k, a.stride, a.L);
  if (n_tiles + extra == 0) return hipSuccess;
  const dim3 grid((unsigned)(n_tiles + extra));
  if (kind == 1) {
    hipLaunchKernelGGL((conv_chans_kernel<kChansC, kChansK>), grid, dim3(kBlock), lds, s, a, (int32_t)n_tiles, extra,
                       fpe, n_ct);
  } else if (kind == 3) {
    if (a.cin == 16)
      hipLaunchKernelGGL((conv_out1_kernel<16, 8>), grid, dim3(kBlock), lds, s, a, (int32_t)n_tiles, extra, fpe);
    else if (a.cin == 32)
      hipLaunchKernelGGL((conv_out1_kernel<32, 8>), grid, dim3(kBlock), lds, s, a, (int32_t)n_tiles, extra, fpe);
    else
      hipLaunchKernelGGL((conv_out1_kernel<48, 8>), grid, dim3(kBlock), lds, s, a, (int32_t)n_tiles, extra, fpe);
  } else {
    hipLaunchKernelGGL(conv_frames_kernel, grid, dim3(kBlock), lds, s, a, (int32_t)n_tiles, extra, fpe);
  }
  return hipGetLastError();
}

hipError_t launch_pack_input(const Entry* ents, const int32_t* fent, int32_t granule, const int32_t* hdr, int32_t C,
                             int64_t max_frames, float* out, void* twin, int32_t twin_prec, int32_t twin_pre,
                             float twin_qs, hipStream_t s) {
  hipLaunchKernelGGL(pack_input_kernel, dim3(grid_for(max_frames * C)), dim3(kBlock), 0, s, ents, fent,
                     make_fastdiv((uint32_t)std::max(granule, 1)), hdr, C, out, twin, twin_prec, twin_pre, twin_qs);
  return hipGetLastError();
}

hipError_t launch_convt_valu(const LayerArgs& a, hipStream_t s) {
  const int64_t items = (a.n_in + a.n_ent) * a.stride * a.cout;
  hipLaunchKernelGGL(convt_valu_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a,
                     make_fastdiv((uint32_t)a.stride));
  return hipGetLastError();
}

hipError_t launch_delay_add(const LayerArgs& a, hipStream_t s) {
  const int64_t items = a.n_out * a.cout + (int64_t)a.n_ent * (a.A0 + a.A1) * a.cout;
  hipLaunchKernelGGL(delay_add_kernel, dim3(grid_for(items)), dim3(kBlock), 0, s, a,
                     make_fastdiv((uint32_t)std::max((a.A0 + a.A1) * a.cout, 1)));
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
