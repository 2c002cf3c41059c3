// Offline evaluation of a model on finite buffers (zero padding at both ends
// of every layer, the non-causal model as trained, Sec. 2.1), and the
// overlap-add baseline the paper compares the streaming method with
// (Sec. 3.3), both on the streaming kernels.
//
// A buffer of T input frames is run through an internal stream whose state
// starts at zero and with both output masks on: the warm-up mask zeroes every
// layer's output before the layer's delay (the left zero padding), the end
// mask zeroes it from the layer's offline length on (the right zero padding),
// so every layer sees exactly the zero-padded input of the offline model.
// The stream is fed the buffer plus F zero frames (F = ceil(D / output rate),
// whole granules), after which its output from sample D on is the offline
// output of the buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "model_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr size_t kAlignFloats = 64;   // 256-byte regions in the offline buffer

size_t align_floats(size_t v) { return (v + kAlignFloats - 1) / kAlignFloats * kAlignFloats; }

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>((n + kBlock - 1) / kBlock, 1), 65535); }

// Input frames after a buffer that bring the streamed output up to the
// buffer's last offline sample.
int64_t flush_frames(const sc::Plan& pl) {
  const int64_t num = pl.out_rate.num, den = pl.out_rate.den, g = pl.input_multiple;
  const int64_t f = (pl.latency * den + num - 1) / num;
  return (f + g - 1) / g * g;
}

// pad[k * stride + c * tp + t] = x[c][k * hop + t] for t < win, 0 for
// win <= t < tp.
__global__ void ola_gather_kernel(const float* __restrict__ x, int64_t n_frames, int32_t C, int32_t K, int64_t win,
                                  int64_t hop, int64_t tp, int64_t stride, float* __restrict__ pad) {
  const int64_t total = (int64_t)K * C * tp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / tp, t = i - row * tp;
    const int64_t k = row / C, c = row - k * C;
    pad[k * stride + c * tp + t] = t < win ? x[c * n_frames + k * hop + t] : 0.f;
  }
}

// Overlap-add of K buffer outputs: out[c][p] = sum over buffers k with
// 0 <= p - k * hop < win of taper(p - k * hop) * Y_k[c][off + p - k * hop],
// in increasing k.  The taper rises as sin^2 over the first `ov` samples,
// is 1 in between and falls as the mirror image over the last `ov`.
__global__ void ola_synth_kernel(const float* __restrict__ Y, int64_t y_stride, int64_t y_pitch, int64_t y_off,
                                 int32_t K, int64_t win, int64_t hop, int64_t ov, int64_t n_out,
                                 float* __restrict__ out) {
  const int c = blockIdx.y;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n_out; p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k_hi = std::min<int64_t>(K - 1, p / hop);
    const int64_t k_lo = p >= win ? (p - win) / hop + 1 : 0;
    float acc = 0.f;
    for (int64_t k = k_lo; k <= k_hi; ++k) {
      const int64_t n = p - k * hop;
      float w = 1.f;
      if (n < ov) {
        const float s = sinpif((float)n / (float)(2 * ov));
        w = s * s;
      } else if (n >= win - ov) {
        const float s = sinpif((float)(win - n) / (float)(2 * ov));
        w = s * s;
      }
      acc += w * Y[k * y_stride + (int64_t)c * y_pitch + y_off + n];
    }
    out[(int64_t)c * n_out + p] = acc;
  }
}

// Sizes the internal streams (n of them, buffers up to max_tp frames) and the
// offline buffer (`floats`), and zeroes the streams' states on hs.
sc_status prepare_offline(sc_model* m, int n, int64_t max_tp, size_t floats, hipStream_t hs) {
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return sc::fail_hip(e, "hipSetDevice");
  const size_t stride = align_floats((size_t)std::max<int64_t>(m->plan.state_alloc_floats, 1));
  if ((int)m->off_streams.size() < n || m->off_cap < floats) {
    // earlier offline work may still read the buffers being replaced
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return sc::fail_hip(e, "hipDeviceSynchronize");
  }
  if ((int)m->off_streams.size() < n) {
    const size_t cap = std::max<size_t>((size_t)n, 2 * m->off_streams.size());
    hipFree(m->off_state);
    m->off_state = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&m->off_state), cap * stride * sizeof(float));
    if (e != hipSuccess) {
      for (sc_stream* s : m->off_streams) delete s;
      m->off_streams.clear();
      return sc::fail_status(SC_ENOMEM, "offline stream state allocation failed");
    }
    while (m->off_streams.size() < cap) {
      sc_stream* s = new (std::nothrow) sc_stream();
      if (!s) return sc::fail_status(SC_ENOMEM, "host allocation failed");
      s->m = m;
      m->off_streams.push_back(s);
    }
    for (size_t i = 0; i < m->off_streams.size(); ++i) m->off_streams[i]->d_state = m->off_state + i * stride;
  }
  if (m->off_cap < floats) {
    const size_t cap = std::max(floats, m->off_cap * 2);
    hipFree(m->off_buf);
    m->off_buf = nullptr;
    m->off_cap = 0;
    e = hipMalloc(reinterpret_cast<void**>(&m->off_buf), cap * sizeof(float));
    if (e != hipSuccess) return sc::fail_status(SC_ENOMEM, "offline buffer allocation failed");
    m->off_cap = cap;
  }
  if (!m->off_done) {
    e = hipEventCreateWithFlags(&m->off_done, hipEventDisableTiming);
    if (e != hipSuccess) return sc::fail_hip(e, "hipEventCreate");
  }
  for (int i = 0; i < n; ++i) {
    sc_stream* s = m->off_streams[i];
    s->max_frames = (int32_t)max_tp;
    s->flags = SC_FLAG_WARMUP_MASK;
    s->pos = 0;
    s->parity = 0;
    s->bad = false;
  }
  if (m->has_last) {
    e = hipStreamWaitEvent(hs, m->last_done, 0);
    if (e != hipSuccess) return sc::fail_hip(e, "hipStreamWaitEvent");
  }
  e = sc::launch_fill_zero(m->off_state, (int64_t)(n * stride), hs);
  if (e != hipSuccess) return sc::fail_hip(e, "state reset");
  return SC_OK;
}

sc_status finish_offline(sc_model* m, hipStream_t hs) {
  const hipError_t e = hipEventRecord(m->off_done, hs);
  if (e != hipSuccess) return sc::fail_hip(e, "hipEventRecord");
  m->last_done = m->off_done;
  m->has_last = true;
  return SC_OK;
}

}  // namespace

extern "C" {

sc_status sc_offline_batch(sc_model* m, int32_t n, const float* const* d_in, const int32_t* n_frames,
                           float* const* d_out, void* hip_stream) {
  if (!m || n <= 0 || !d_in || !n_frames || !d_out) return sc::fail_status(SC_EINVAL, "null argument or n <= 0");
  std::lock_guard<std::mutex> g(m->mu);
  const sc::Plan& pl = m->plan;
  const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
  const int64_t F = flush_frames(pl);
  std::vector<int32_t> tp(n);
  std::vector<size_t> in_off(n), out_off(n);
  size_t floats = 0;
  int64_t max_tp = 0;
  for (int i = 0; i < n; ++i) {
    if (!d_in[i] || !d_out[i]) return sc::fail_status(SC_EINVAL, "null device buffer");
    const int64_t T = n_frames[i];
    if (T < 1 || T % pl.input_multiple != 0 || T + F > INT32_MAX / 4)
      return sc::fail_status(SC_ELENGTH, "buffer length must be >= 1 and a multiple of the total stride");
    tp[i] = (int32_t)(T + F);
    max_tp = std::max<int64_t>(max_tp, tp[i]);
    in_off[i] = floats;
    floats += align_floats((size_t)pl.in_channels * tp[i]);
    out_off[i] = floats;
    floats += align_floats((size_t)pl.out_channels * pl.out_rate.of(tp[i]));
  }
  sc_status st = prepare_offline(m, n, max_tp, floats, hs);
  if (st != SC_OK) return st;
  std::vector<const float*> ins(n);
  std::vector<float*> outs(n);
  for (int i = 0; i < n; ++i) {
    m->off_streams[i]->end = n_frames[i];
    ins[i] = m->off_buf + in_off[i];
    outs[i] = m->off_buf + out_off[i];
  }
  // the padded inputs: the buffer, then F zero frames per channel
  hipError_t e = hipSuccess;
  for (int i = 0; e == hipSuccess && i < n; ++i) {
    float* pad = m->off_buf + in_off[i];
    e = sc::launch_fill_zero(pad, (int64_t)pl.in_channels * tp[i], hs);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(pad, (size_t)tp[i] * sizeof(float), d_in[i], (size_t)n_frames[i] * sizeof(float),
                           (size_t)n_frames[i] * sizeof(float), (size_t)pl.in_channels, hipMemcpyDeviceToDevice, hs);
  }
  if (e != hipSuccess) return sc::fail_hip(e, "offline input staging");
  st = sc::run_step_locked(m, n, m->off_streams.data(), ins.data(), tp.data(), outs.data(), hs);
  for (int i = 0; i < n; ++i) m->off_streams[i]->end = 0;
  if (st != SC_OK) return st;
  // the offline output of buffer i is its streamed output from sample D on
  for (int i = 0; e == hipSuccess && i < n; ++i) {
    const int64_t w = pl.out_rate.of(n_frames[i]), wp = pl.out_rate.of(tp[i]);
    e = hipMemcpy2DAsync(d_out[i], (size_t)w * sizeof(float), outs[i] + pl.latency, (size_t)wp * sizeof(float),
                         (size_t)w * sizeof(float), (size_t)pl.out_channels, hipMemcpyDeviceToDevice, hs);
  }
  if (e != hipSuccess) return sc::fail_hip(e, "offline output copy");
  return finish_offline(m, hs);
}

sc_status sc_ola_process(sc_model* m, const float* d_in, int32_t n_frames, int32_t window, int32_t overlap,
                         float* d_out, void* hip_stream) {
  if (!m || !d_in || !d_out) return sc::fail_status(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(m->mu);
  const sc::Plan& pl = m->plan;
  const hipStream_t hs = static_cast<hipStream_t>(hip_stream);
  const int64_t gm = pl.input_multiple;
  if (n_frames < 1 || n_frames % gm != 0 || window < 1 || window % gm != 0 || overlap < 0 || overlap % gm != 0 ||
      2 * (int64_t)overlap > window)
    return sc::fail_status(SC_ELENGTH, "lengths must be whole granules, overlap at most half the window");
  const int64_t hop = window - overlap;
  const int64_t K = n_frames >= window ? (n_frames - window) / hop + 1 : 0;
  const int64_t F = flush_frames(pl);
  const int64_t tp = window + F;
  const int64_t n_out = pl.out_rate.of(n_frames);
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return sc::fail_hip(e, "hipSetDevice");
  if (K == 0) {
    // no complete buffer: the baseline has produced nothing yet
    e = sc::launch_fill_zero(d_out, (int64_t)pl.out_channels * n_out, hs);
    return e == hipSuccess ? SC_OK : sc::fail_hip(e, "output fill");
  }
  if (tp > INT32_MAX / 4 || K > INT32_MAX / 4 || K * tp > INT32_MAX / 4)
    return sc::fail_status(SC_ELENGTH, "signal too long for one call");
  const size_t in_stride = align_floats((size_t)pl.in_channels * tp);
  const int64_t out_tp = pl.out_rate.of(tp);
  const size_t out_stride = align_floats((size_t)pl.out_channels * out_tp);
  const size_t out_base = (size_t)K * in_stride;
  sc_status st = prepare_offline(m, (int)K, tp, out_base + (size_t)K * out_stride, hs);
  if (st != SC_OK) return st;
  std::vector<const float*> ins(K);
  std::vector<float*> outs(K);
  std::vector<int32_t> tps(K, (int32_t)tp);
  for (int64_t k = 0; k < K; ++k) {
    m->off_streams[k]->end = window;
    ins[k] = m->off_buf + (size_t)k * in_stride;
    outs[k] = m->off_buf + out_base + (size_t)k * out_stride;
  }
  hipLaunchKernelGGL(ola_gather_kernel, dim3(grid_for(K * pl.in_channels * tp)), dim3(kBlock), 0, hs, d_in,
                     (int64_t)n_frames, pl.in_channels, (int32_t)K, (int64_t)window, hop, tp, (int64_t)in_stride,
                     m->off_buf);
  e = hipGetLastError();
  if (e != hipSuccess) return sc::fail_hip(e, "overlap-add input staging");
  st = sc::run_step_locked(m, (int)K, m->off_streams.data(), ins.data(), tps.data(), outs.data(), hs);
  for (int64_t k = 0; k < K; ++k) m->off_streams[k]->end = 0;
  if (st != SC_OK) return st;
  hipLaunchKernelGGL(ola_synth_kernel, dim3(grid_for(n_out), (unsigned)pl.out_channels), dim3(kBlock), 0, hs,
                     m->off_buf + out_base, (int64_t)out_stride, out_tp, pl.latency, (int32_t)K,
                     pl.out_rate.of(window), pl.out_rate.of(hop), pl.out_rate.of(overlap), n_out, d_out);
  e = hipGetLastError();
  if (e != hipSuccess) return sc::fail_hip(e, "overlap-add synthesis");
  return finish_offline(m, hs);
}

}  // extern "C"
