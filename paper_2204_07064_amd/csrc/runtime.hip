// Runtime and C ABI: models (plan + device weights), streams (device state),
// batched processing steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

#include "kernels.h"
#include "model_internal.h"
#include "sc_internal.h"

namespace sc {

namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error_cstr() { return g_err.c_str(); }

}  // namespace sc

using namespace sc;

namespace {

sc_status fail(sc_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

sc_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return SC_EDEVICE;
}

}  // namespace

namespace {

// Packs a conv's W[co][ci][k] into [k][ci][co] (FP32 wavefront kernels).
std::vector<float> pack_conv_valu(const float* w, int cout, int cin, int k) {
  std::vector<float> p((size_t)cout * cin * k);
  for (int co = 0; co < cout; ++co)
    for (int ci = 0; ci < cin; ++ci)
      for (int kk = 0; kk < k; ++kk) p[((size_t)kk * cin + ci) * cout + co] = w[((size_t)co * cin + ci) * k + kk];
  return p;
}

// Packs a transposed conv's W[ci][co][2r] into [h][phi][ci][co] with
// h = 0 -> tap phi + r (previous frame), h = 1 -> tap phi (current frame).
std::vector<float> pack_convt_valu(const float* w, int cin, int cout, int r) {
  std::vector<float> p((size_t)2 * r * cin * cout);
  for (int h = 0; h < 2; ++h)
    for (int phi = 0; phi < r; ++phi)
      for (int ci = 0; ci < cin; ++ci)
        for (int co = 0; co < cout; ++co) {
          const int tap = h == 0 ? phi + r : phi;
          p[(((size_t)h * r + phi) * cin + ci) * cout + co] = w[((size_t)ci * cout + co) * (2 * r) + tap];
        }
  return p;
}

template <class T>
hipError_t upload(T** dst, const T* src, size_t n) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

void free_model(sc_model* m) {
  if (!m) return;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  for (auto& o : m->opdev) {
    hipFree(o.W);
    hipFree(o.B);
    hipFree(o.wscale);
  }
  for (float* p : m->ws) hipFree(p);
  for (void* p : m->tw) hipFree(p);
  for (hipEvent_t ev : m->prof_events) hipEventDestroy(ev);
  for (auto& s : m->ring) {
    if (s.host) hipHostFree(s.host);
    if (s.dev) hipFree(s.dev);
    if (s.done) hipEventDestroy(s.done);
  }
  if (m->own_done) hipEventDestroy(m->own_done);
  if (m->side) {
    hipStreamSynchronize(m->side);
    hipStreamDestroy(m->side);
  }
  if (m->fork_ev) hipEventDestroy(m->fork_ev);
  if (m->join_ev) hipEventDestroy(m->join_ev);
  if (m->graph_exec) hipGraphExecDestroy(m->graph_exec);
  hipFree(m->graph_desc);
  if (m->capture_stream) hipStreamDestroy(m->capture_stream);
  hipFree(m->d_amax);
  for (sc_stream* s : m->off_streams) delete s;   // their states live in off_state
  hipFree(m->off_state);
  hipFree(m->off_buf);
  if (m->off_done) hipEventDestroy(m->off_done);
  delete m;
}

// Scale applied before rounding a twin read by `layer`: the reciprocal of that
// layer's FP8 activation scale (amax / 448), computed as the MFMA kernel does.
float twin_scale(const sc_model* m, int layer) {
  if (layer < 0 || m->layer_prec[layer] != 2 || !m->have_scales) return 1.0f;
  return 1.0f / (m->act_scales[layer] / 448.0f);
}

// Workspace buffer b / operand twin t from input frame `base` on.
float* ws_at(const sc_model* m, const WsView& w, int b, int64_t base) {
  return b >= 0 ? w.ws[b] + m->plan.buf_floats[b].of(base) : nullptr;
}
void* tw_at(const sc_model* m, const WsView& w, int t, int64_t base) {
  return t >= 0 ? static_cast<unsigned char*>(w.tw[t]) + m->plan.twin_elems[t].of(base) * m->plan.twin_esize[t]
                : nullptr;
}

// A one-output-channel stride-1 conv that writes the model output and reads
// only the output of the window conv launched just before it, which nothing
// else reads, is computed in that conv's epilogue (IMPL_TAIL).
void fuse_output_convs(Plan& pl) {
  for (size_t i = 1; i < pl.ops.size(); ++i) {
    Op& c = pl.ops[i];
    Op& p = pl.ops[i - 1];
    if (c.kind != K_CONV || c.impl != IMPL_VALU || c.cout != 1 || c.stride != 1 || c.out_buf != -1 ||
        c.residual || c.in_buf2 >= 0 || (c.post_act != 0 && c.post_act != 2))
      continue;
    if (p.kind != K_CONV || p.impl != IMPL_WIN || p.out_buf < 0 || c.in_buf != p.out_buf || p.fuse_out >= 0)
      continue;
    if (c.cache_len != c.dil * (c.k - 1) || !conv_win_out_fusable(p.cin, p.cout, c.k, c.dil)) continue;
    // (workspace buffers are reused, so readers are found by node)
    bool other = false;
    for (size_t j = 0; j < pl.ops.size(); ++j)
      if (j != i && (pl.ops[j].src == p.node || pl.ops[j].src2 == p.node)) other = true;
    if (other) continue;
    p.fuse_out = (int32_t)i;
    c.fuse_out = (int32_t)(i - 1);
    c.impl = IMPL_TAIL;
  }
}

// A transposed conv whose output only a residual window conv reads (the
// first residual block of a narrow stage) runs inside that conv's launch
// (launch_convt_win), where the tiles compute the frames their windows need;
// both ops then share one launch and the transposed conv's output is never
// written.  It needs the transposed conv to read its input in operand form.
// The model input read straight from the callers' channel-major buffers by
// its only reader, an FP32 MFMA conv (no residual, no operand copy of the
// input): the packing launch goes away.
void mark_input_direct(sc_model* m) {
  Plan& pl = m->plan;
  if (pl.input_buf < 0 || pl.input_twin >= 0) return;
  int reader = -1, readers = 0;
  for (size_t o = 0; o < pl.ops.size(); ++o) {
    const Op& op = pl.ops[o];
    const int r = (op.src == 0) + (op.src2 == 0);
    if (r) reader = (int)o;
    readers += r;
  }
  if (readers != 1) return;
  Op& op = pl.ops[reader];
  // (the 64-row tile the gathering kernel uses for more than 32 output channels)
  if (op.kind != K_CONV || op.impl != IMPL_MFMA || op.prec != 0 || op.residual || op.in_twin >= 0 ||
      op.cin % 4 != 0 || op.cout <= 32)
    return;
  op.user_in = 1;
  m->input_direct = true;
}

void fuse_convt_windows(sc_model* m) {
  Plan& pl = m->plan;
  for (size_t w = 0; w < pl.ops.size(); ++w) {
    Op& cv = pl.ops[w];
    if (cv.kind != K_CONV || cv.impl != IMPL_WIN || !cv.residual || cv.fuse_out >= 0 || cv.prec < 1) continue;
    int c = -1, readers = 0;
    for (size_t o = 0; o < pl.ops.size(); ++o) {
      if (pl.ops[o].node == cv.src) c = (int)o;
      readers += (pl.ops[o].src == cv.src) + (pl.ops[o].src2 == cv.src);
    }
    if (c < 0 || readers != 1) continue;
    Op& ct = pl.ops[c];
    if (ct.kind != K_CONVT || ct.impl != IMPL_MFMA || ct.in_twin < 0 || ct.prec != cv.prec || ct.out_twin >= 0)
      continue;
    const int64_t min_frames = cv.in_rate.of(pl.input_multiple);
    int32_t xrows = 0, stash = 0;
    const int32_t rows = convt_win_rows(cv.cin, cv.cout, cv.k, cv.dil, cv.cache_len, ct.stride, ct.cin, cv.prec,
                                        min_frames, &xrows, &stash);
    if (rows <= 0) continue;
    cv.convt_in = c;
    ct.convt_in = (int32_t)w;
    m->opdev[w].ct_rows = rows;
    m->opdev[w].ct_xrows = xrows;
    m->opdev[w].ct_stash = stash;
  }
}

// Two residual window convs launched one after the other, the second the
// first's only reader (consecutive residual blocks of a 64-channel stage),
// share one launch (launch_conv_pair): the second conv's tiles compute the
// frames of the first one's output that their windows need, and that output
// is never formed.  Pairs are taken greedily in order (blocks 1 + 2 of a
// stack).  Such a model runs pairs fused always (activation maxima, which
// need the first conv's output, are refused on it).
bool pair_candidate(const Op& op) {
  return op.kind == K_CONV && op.impl == IMPL_WIN && op.residual && op.convt_in < 0 && op.stride == 1 &&
         op.cin == op.cout && op.prec >= 1;
}

void fuse_conv_pairs(sc_model* m) {
  Plan& pl = m->plan;
  for (size_t b = 0; b < pl.ops.size(); ++b) {
    Op& cb = pl.ops[b];
    // (the pair writes its output to a workspace buffer: not the model output)
    if (!pair_candidate(cb) || cb.in_twin >= 0 || cb.out_buf < 0) continue;
    int ia = -1, readers = 0;
    for (size_t o = 0; o < pl.ops.size(); ++o) {
      if (pl.ops[o].node == cb.src) ia = (int)o;
      readers += (pl.ops[o].src == cb.src) + (pl.ops[o].src2 == cb.src);
    }
    if (ia < 0 || ia + 1 != (int)b || readers != 1) continue;
    Op& ca = pl.ops[ia];
    // (the first conv of a pair computes no output conv in its epilogue; the
    // second may)
    if (!pair_candidate(ca) || ca.fuse_out >= 0 || ca.pair_in >= 0 || ca.pair_out >= 0 || ca.out_twin >= 0 ||
        ca.prec != cb.prec || ca.k != cb.k || ca.cin != cb.cin)
      continue;
    const int64_t min_frames = cb.in_rate.of(pl.input_multiple);
    int32_t arows = 0, stash = 0;
    const int32_t rows =
        conv_pair_rows(cb.cin, cb.k, ca.dil, cb.dil, cb.prec, min_frames, cb.fuse_out >= 0, &arows, &stash);
    if (rows <= 0) continue;
    cb.pair_in = ia;
    ca.pair_out = (int32_t)b;
    ++m->n_pairs;
    // The launch reads A's input while its tiles write B's output.  Where the
    // planner reused A's input buffer for B's output (A was its last reader),
    // B's output takes A's output buffer instead -- never written now -- and
    // the two buffers trade places in every later op (both are free between
    // A and B, and hold the same sizes); else B's output and its readers move
    // to a buffer of their own.
    if (cb.out_buf >= 0 && cb.out_buf == ca.in_buf) {
      const int32_t P = ca.in_buf, Q = ca.out_buf;
      if (Q >= 0 && pl.buf_floats[P].num == pl.buf_floats[Q].num && pl.buf_floats[P].den == pl.buf_floats[Q].den) {
        auto trade = [P, Q](int32_t& x) { x = x == P ? Q : (x == Q ? P : x); };
        for (size_t o = b; o < pl.ops.size(); ++o) {
          trade(pl.ops[o].in_buf);
          trade(pl.ops[o].in_buf2);
          trade(pl.ops[o].out_buf);
        }
      } else {
        const int32_t nb = (int32_t)pl.buf_floats.size();
        pl.buf_floats.push_back(pl.buf_floats[cb.out_buf]);
        for (Op& o : pl.ops) {
          if (o.src == cb.node) o.in_buf = nb;
          if (o.src2 == cb.node) o.in_buf2 = nb;
        }
        cb.out_buf = nb;
      }
    }
    m->opdev[b].pair_rows = rows;
    m->opdev[b].pair_arows = arows;
    m->opdev[b].pair_stash = stash;
  }
}

LayerArgs layer_args(const sc_model* m, const Op& op, const Entry* dents, const int32_t* dfent,
                     const int32_t* dhdr, int n_ent, int64_t total_T, int64_t base, const WsView& w) {
  LayerArgs a{};
  a.ents = dents;
  a.fent = dfent;
  a.hdr = dhdr;
  a.n_ent = n_ent;
  a.in_buf = ws_at(m, w, op.in_buf, base);
  a.in_buf2 = ws_at(m, w, op.in_buf2, base);
  a.out_buf = ws_at(m, w, op.out_buf, base);
  const size_t oi = &op - &m->plan.ops[0];
  a.W = m->opdev[oi].W;
  a.B = m->opdev[oi].B;
  a.wscale = m->opdev[oi].wscale;
  a.act_scale = (op.layer >= 0 && m->have_scales) ? m->act_scales[op.layer] / 448.0f : 1.0f;
  a.cin = op.cin; a.cout = op.cout; a.k = op.k; a.dil = op.dil; a.stride = op.stride;
  a.L = op.cache_len; a.pre_act = op.pre_act; a.post_act = op.post_act;
  a.residual = op.residual; a.skip_off = op.skip_off;
  a.A0 = op.A0; a.A1 = op.A1;
  a.in_num = (uint32_t)op.in_rate.num; a.in_den = (uint32_t)op.in_rate.den;
  a.out_num = (uint32_t)op.out_rate.num; a.out_den = (uint32_t)op.out_rate.den;
  // the step's frame table has one entry per input_multiple input frames
  a.fd_in_num = make_fastdiv(a.in_num * (uint32_t)m->plan.input_multiple);
  a.fd_in_den = make_fastdiv(a.in_den);
  a.fd_out_num = make_fastdiv(a.out_num * (uint32_t)m->plan.input_multiple);
  a.fd_out_den = make_fastdiv(a.out_den);
  a.fd_cin = make_fastdiv((uint32_t)std::max(op.cin, 1));
  a.fd_cout = make_fastdiv((uint32_t)std::max(op.cout, 1));
  a.fd_per_ent_narrow = make_fastdiv((uint32_t)std::max(op.cache_len * op.cin, 1));
  a.delay = op.out_delay;
  a.state_off = op.state_off; a.state_len = op.state_len;
  a.state_off2 = op.state_off2; a.state_len2 = op.state_len2;
  a.n_in = op.in_rate.of(total_T);
  a.n_out = op.out_rate.of(total_T);
  a.tile = (op.kind == K_CONV && (op.impl == IMPL_VALU || op.impl == IMPL_TAIL))
               ? narrow_conv_tile(op.cin, op.cout, op.k, op.dil, op.stride, op.cache_len, a.n_out)
               : 0;
  a.in_twin = tw_at(m, w, op.in_twin, base);
  a.out_twin = tw_at(m, w, op.out_twin, base);
  a.twin_prec = op.twin_prec;
  a.twin_pre = op.twin_pre;
  // calibration reads every layer's FP32 input, so keep writing it then
  a.twin_only = (op.twin_only && a.out_twin && !m->amax_on) ? 1 : 0;
  // calibration reads the packed input, so it is packed then
  a.user_in = (op.user_in && !m->amax_on) ? 1 : 0;
  a.twin_qs = twin_scale(m, op.twin_layer);
  a.tstate_off = op.tstate_off;
  a.tstate_len = op.tstate_len;
  return a;
}

}  // namespace

namespace {

// The largest per-launch item count (outputs, transposed-conv columns times
// phases, cache and delay-line items) of a step of n streams and T input
// frames.  Kernels index items in 32-bit integers with grid-stride loops, so
// a step is refused when this exceeds half the int32 range.
int64_t max_step_items(const Plan& pl, int64_t n, int64_t T) {
  int64_t worst = 0;
  for (const Op& op : pl.ops) {
    const int64_t in = op.in_rate.of(T), out = op.out_rate.of(T);
    int64_t v = in * op.cin;
    v = std::max(v, out * op.cout + n * ((int64_t)op.cache_len * op.cin + (int64_t)(op.A0 + op.A1) * op.cout));
    if (op.kind == K_CONVT) v = std::max(v, (in + n) * op.stride * op.cout);
    worst = std::max(worst, v);
  }
  return worst;
}
constexpr int64_t kMaxStepItems = INT32_MAX / 2;

}  // namespace

sc_status sc::ensure_workspace(sc_model* m, int64_t frames) {
  if (frames <= m->ws_cap) return SC_OK;
  // every stream brings at least one granule of input frames
  if (max_step_items(m->plan, frames / m->plan.input_multiple + 1, frames) > kMaxStepItems)
    return fail(SC_ELENGTH, "step too large for 32-bit item indexing");
  if (m->ws_pins > 0)
    return fail(SC_ELENGTH, "step larger than the workspace that a server's captured graph holds");
  int64_t cap = std::max<int64_t>(frames, 2 * m->ws_cap);
  const int64_t mult = m->plan.input_multiple;
  cap = (cap + mult - 1) / mult * mult;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  if (m->graph_exec) {   // captured with the old addresses
    hipGraphExecDestroy(m->graph_exec);
    m->graph_exec = nullptr;
  }
  for (float*& p : m->ws) { hipFree(p); p = nullptr; }
  for (void*& p : m->tw) { hipFree(p); p = nullptr; }
  m->ws.assign(m->plan.buf_floats.size(), nullptr);
  m->tw.assign(m->plan.twin_elems.size(), nullptr);
  for (size_t t = 0; t < m->plan.twin_elems.size(); ++t) {
    const int64_t bytes = m->plan.twin_elems[t].of(cap) * m->plan.twin_esize[t] + 64;
    e = hipMalloc(&m->tw[t], (size_t)bytes);
    if (e != hipSuccess) {
      m->ws_cap = 0;
      return fail(SC_ENOMEM, "workspace allocation failed");
    }
  }
  for (size_t b = 0; b < m->plan.buf_floats.size(); ++b) {
    const int64_t n = m->plan.buf_floats[b].of(cap) + 1;
    e = hipMalloc(reinterpret_cast<void**>(&m->ws[b]), (size_t)n * sizeof(float));
    if (e != hipSuccess) {
      m->ws_cap = 0;
      return fail(SC_ENOMEM, "workspace allocation failed");
    }
  }
  m->ws_cap = cap;
  return SC_OK;
}

namespace {

// Records the start event of a timed launch and hands out its end event.
hipError_t prof_begin(sc_model* m, int oi, const LayerArgs& a, hipStream_t hs, hipEvent_t* ev_end) {
  while (m->prof_events.size() < m->prof_used + 2) {
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return e;
    m->prof_events.push_back(ev);
  }
  hipEvent_t b = m->prof_events[m->prof_used];
  *ev_end = m->prof_events[m->prof_used + 1];
  m->prof_used += 2;
  m->prof_op.push_back(oi);
  m->prof_in.push_back(a.n_in);
  m->prof_out.push_back(a.n_out);
  m->prof_ent.push_back(a.n_ent);
  return hipEventRecord(b, hs);
}

// Waits for the recorded events and adds their durations to the per-op sums.
hipError_t prof_fold(sc_model* m) {
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < m->prof_op.size(); ++i) {
    e = hipEventSynchronize(m->prof_events[2 * i + 1]);
    if (e != hipSuccess) break;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, m->prof_events[2 * i], m->prof_events[2 * i + 1]);
    if (e != hipSuccess) break;
    sc_op_profile& p = m->prof[m->prof_op[i]];
    p.ms += ms;
    p.launches += 1;
    p.frames_in += m->prof_in[i];
    p.frames_out += m->prof_out[i];
    p.entries += m->prof_ent[i];
  }
  m->prof_used = 0;
  m->prof_op.clear();
  m->prof_in.clear();
  m->prof_out.clear();
  m->prof_ent.clear();
  return e;
}

}  // namespace

namespace sc {

sc_status fail_status(sc_status st, const char* msg) { return fail(st, msg); }

sc_status validate_step(sc_model* m, int n, sc_stream* const* streams, const float* const* d_in,
                        const int32_t* n_frames, float* const* d_out, int64_t* total_out) {
  if (n <= 0 || !streams || !d_in || !n_frames || !d_out) return fail(SC_EINVAL, "null argument or n <= 0");
  if (m->any_fp8 && !m->have_scales) return fail(SC_EINVAL, "FP8 model has no activation scales");
  int64_t total = 0;
  const uint64_t gen = ++m->step_gen;
  for (int i = 0; i < n; ++i) {
    sc_stream* s = streams[i];
    if (!s || s->m != m) return fail(SC_EINVAL, "stream is null or belongs to another model");
    if (s->seen == gen) return fail(SC_EINVAL, "a stream appears twice in one batch");
    s->seen = gen;
    if (s->bad) return fail(SC_ESTATE, "stream saw a device error; call stream_reset");
    const int32_t T = n_frames[i];
    if (T < 1 || T > s->max_frames || T % m->plan.input_multiple != 0)
      return fail(SC_ELENGTH, "buffer length must be in [1, max_buffer_frames] and a multiple of the total stride");
    if (!d_in[i] || !d_out[i]) return fail(SC_EINVAL, "null device buffer");
    total += T;
  }
  if (total > INT32_MAX / 4 || max_step_items(m->plan, n, total) > kMaxStepItems)
    return fail(SC_ELENGTH, "batch too large for 32-bit item indexing");
  *total_out = total;
  return SC_OK;
}

void fill_descriptor(unsigned char* host, int n, int ent_capacity, sc_stream* const* streams,
                     const float* const* d_in, const int32_t* n_frames, float* const* d_out, int64_t total,
                     int64_t granule) {
  int32_t* hhdr = reinterpret_cast<int32_t*>(host);
  hhdr[0] = n;
  hhdr[1] = (int32_t)total;
  Entry* hents = reinterpret_cast<Entry*>(host + kDescHeaderBytes);
  int32_t* hfent = reinterpret_cast<int32_t*>(host + kDescHeaderBytes + (size_t)ent_capacity * sizeof(Entry));
  int32_t off = 0;
  for (int i = 0; i < n; ++i) {
    Entry& en = hents[i];
    en.in = d_in[i];
    en.out = d_out[i];
    en.state = streams[i]->d_state;
    en.T = n_frames[i];
    en.off = off;
    en.parity = streams[i]->parity;
    en.flags = (int32_t)streams[i]->flags;
    en.pos = streams[i]->pos;
    en.end = streams[i]->end;
    for (int32_t f = 0; f < n_frames[i]; f += (int32_t)granule) hfent[(off + f) / granule] = i;
    off += n_frames[i];
  }
}

namespace {

// One launch set: a step's (or a split step half's) descriptor on the device,
// its grid bounds, stream and workspace offset.
struct LaunchSet {
  const int32_t* hdr;
  const Entry* ents;
  const int32_t* fent;
  int grid_n;
  int64_t grid_frames;
  hipStream_t hs;
  int64_t base;
  WsView w;
};

LaunchSet launch_set(const unsigned char* dev, int grid_n, int64_t grid_frames, hipStream_t hs, int64_t base,
                     const WsView& w) {
  LaunchSet ls;
  ls.w = w;
  ls.hdr = reinterpret_cast<const int32_t*>(dev);
  ls.ents = reinterpret_cast<const Entry*>(dev + kDescHeaderBytes);
  ls.fent = reinterpret_cast<const int32_t*>(dev + kDescHeaderBytes + (size_t)grid_n * sizeof(Entry));
  ls.grid_n = grid_n;
  ls.grid_frames = grid_frames;
  ls.hs = hs;
  ls.base = base;
  return ls;
}

hipError_t launch_pack(sc_model* m, const LaunchSet& ls) {
  const Plan& pl = m->plan;
  if (pl.input_buf < 0 || (m->input_direct && !m->amax_on)) return hipSuccess;
  return launch_pack_input(ls.ents, ls.fent, pl.input_multiple, ls.hdr, pl.in_channels, ls.grid_frames,
                           ws_at(m, ls.w, pl.input_buf, ls.base),
                           tw_at(m, ls.w, pl.input_twin, ls.base), pl.input_twin_prec,
                           pl.input_twin_pre, twin_scale(m, pl.input_twin_layer), ls.hs);
}

// The one-output-channel conv computed in the epilogue of window conv `op`.
void set_out_conv(const sc_model* m, const Op& op, LayerArgs& aw) {
  const Op& oc = m->plan.ops[op.fuse_out];
  aw.oc.W = static_cast<const float*>(m->opdev[op.fuse_out].W);
  aw.oc.B = m->opdev[op.fuse_out].B;
  aw.oc.k = oc.k;
  aw.oc.dil = oc.dil;
  aw.oc.L = oc.cache_len;
  aw.oc.pre_act = oc.pre_act;
  aw.oc.post_act = oc.post_act;
  aw.oc.delay = oc.out_delay;
  aw.oc.state_off = oc.state_off;
  aw.oc.state_len = oc.state_len;
}

// The launch of op `oi` (with its calibration and timing records, if on).
hipError_t launch_op(sc_model* m, size_t oi, const LaunchSet& ls) {
  const Op& op = m->plan.ops[oi];
  const LayerArgs a = layer_args(m, op, ls.ents, ls.fent, ls.hdr, ls.grid_n, ls.grid_frames, ls.base, ls.w);
  hipError_t e = hipSuccess;
  if (m->amax_on && op.layer >= 0) {
    e = launch_amax(a, m->d_amax + op.layer, ls.hs);
    if (e != hipSuccess) return e;
  }
  const int prec = m->opdev[oi].prec;
  // a transposed conv computed in the launch of the window conv after it
  // (calibration reads its output, so it runs on its own then)
  const bool ct_fused = op.convt_in >= 0 && !m->amax_on;
  if (ct_fused && op.kind == K_CONVT) return hipSuccess;
  // a residual conv computed in the launch of the residual conv after it
  // (always: the model refuses activation maxima, see fuse_conv_pairs)
  if (op.pair_out >= 0) return hipSuccess;
  const bool pair = op.pair_in >= 0;
  hipEvent_t ev_end = nullptr;
  if (m->prof_on) {
    e = prof_begin(m, (int)oi, a, ls.hs, &ev_end);
    if (e != hipSuccess) return e;
  }
  // calibration reads the fused output conv's input, so run it on its own then
  const bool fused = op.fuse_out >= 0 && !m->amax_on;
  if (op.kind == K_CONV) {
    if (op.impl == IMPL_WIN && ct_fused) {
      const Op& ct = m->plan.ops[op.convt_in];
      const OpDev& cd = m->opdev[op.convt_in];
      LayerArgs aw = a;
      aw.ct.W = cd.W;
      aw.ct.B = cd.B;
      aw.ct.wscale = cd.wscale;
      aw.ct.act_scale = (ct.layer >= 0 && m->have_scales) ? m->act_scales[ct.layer] / 448.0f : 1.0f;
      aw.ct.in_twin = tw_at(m, ls.w, ct.in_twin, ls.base);
      aw.ct.r = ct.stride;
      aw.ct.cin = ct.cin;
      const int kc = prec == 1 ? 64 : 128;
      aw.ct.half_pad = (ct.cin + kc - 1) / kc * kc;
      aw.ct.Kpad = 2 * aw.ct.half_pad;
      aw.ct.in_num = (uint32_t)ct.in_rate.num;
      aw.ct.in_den = (uint32_t)ct.in_rate.den;
      aw.ct.fd_in_den = make_fastdiv(aw.ct.in_den);
      aw.ct.delay = ct.out_delay;
      aw.ct.state_off = ct.state_off;
      aw.ct.state_len = ct.state_len;
      e = launch_convt_win(aw, prec, m->opdev[oi].ct_rows, m->opdev[oi].ct_xrows, m->opdev[oi].ct_stash, ls.hs);
    } else if (op.impl == IMPL_WIN && pair) {
      const Op& pa = m->plan.ops[op.pair_in];
      const OpDev& pd = m->opdev[op.pair_in];
      LayerArgs aw = a;
      aw.pa.W = pd.W;
      aw.pa.B = pd.B;
      aw.pa.wscale = pd.wscale;
      aw.pa.act_scale = (pa.layer >= 0 && m->have_scales) ? m->act_scales[pa.layer] / 448.0f : 1.0f;
      aw.pa.in_buf = ws_at(m, ls.w, pa.in_buf, ls.base);
      aw.pa.L = pa.cache_len;
      aw.pa.dil = pa.dil;
      aw.pa.skip_off = pa.skip_off;
      aw.pa.pre_act = pa.pre_act;
      aw.pa.delay = pa.out_delay;
      aw.pa.state_off = pa.state_off;
      aw.pa.state_len = pa.state_len;
      if (op.fuse_out >= 0) set_out_conv(m, op, aw);
      const OpDev& od = m->opdev[oi];
      e = launch_conv_pair(aw, prec, od.pair_rows, od.pair_arows, od.pair_stash, ls.hs);
    } else if (op.impl == IMPL_WIN) {
      LayerArgs aw = a;
      if (fused) set_out_conv(m, op, aw);
      e = launch_conv_win(aw, prec, m->opdev[oi].win_rows, ls.hs);
    } else if (op.impl == IMPL_TAIL && fused) {
      const Op& pw = m->plan.ops[op.fuse_out];
      e = launch_conv_out_tail(a, conv_win_tile_frames(pw.cin, pw.cout), ls.hs);
    } else {
      e = (op.impl == IMPL_MFMA) ? launch_conv_mfma(a, prec, ls.hs) : launch_conv_valu(a, ls.hs);
    }
  } else if (op.kind == K_CONVT) {
    e = (op.impl == IMPL_MFMA) ? launch_convt_mfma(a, prec, ls.hs) : launch_convt_valu(a, ls.hs);
  } else {
    e = launch_delay_add(a, ls.hs);
  }
  if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, ls.hs);
  return e;
}

}  // namespace

hipError_t enqueue_kernels(sc_model* m, const unsigned char* dev, int grid_n, int64_t grid_frames, hipStream_t hs,
                           int64_t base) {
  return enqueue_kernels_ws(m, dev, grid_n, grid_frames, hs, base, model_ws(m));
}

hipError_t enqueue_kernels_ws(sc_model* m, const unsigned char* dev, int grid_n, int64_t grid_frames, hipStream_t hs,
                              int64_t base, const WsView& w) {
  const LaunchSet ls = launch_set(dev, grid_n, grid_frames, hs, base, w);
  hipError_t e = launch_pack(m, ls);
  for (size_t oi = 0; e == hipSuccess && oi < m->plan.ops.size(); ++oi) e = launch_op(m, oi, ls);
  return e;
}

// Where a step splits into two halves of its streams that run at once (the
// kernels are latency-bound, so two half-size launch sequences overlap each
// other's waits): the first `*h` streams with `*f` input frames, the rest
// after them in the workspace.  0 = run the step as one sequence.
int choose_split(const sc_model* m, int n, const int32_t* n_frames, int64_t total, int64_t* f) {
  constexpr int kSplitMinStreams = 32;
  constexpr int64_t kSplitMinFrames = 512;
  if ((m->options & SC_MODEL_NO_SPLIT) || n < kSplitMinStreams || total < kSplitMinFrames) return 0;
  int64_t acc = 0;
  int h = 0;
  while (h < n - 1 && 2 * acc < total) acc += n_frames[h++];
  if (h == 0 || h >= n) return 0;
  // the second half's workspace offsets must be whole and keep 16-byte alignment
  for (const sc::Frac& r : m->plan.buf_floats)
    if (acc * r.num % r.den != 0 || r.of(acc) * (int64_t)sizeof(float) % 16 != 0) return 0;
  for (size_t t = 0; t < m->plan.twin_elems.size(); ++t) {
    const sc::Frac& r = m->plan.twin_elems[t];
    if (acc * r.num % r.den != 0 || r.of(acc) * m->plan.twin_esize[t] % 16 != 0) return 0;
  }
  *f = acc;
  return h;
}

size_t split_desc_offset(int h, int64_t fa, int64_t granule) { return (desc_bytes(h, fa, granule) + 255) / 256 * 256; }

hipError_t enqueue_split(sc_model* m, const unsigned char* dev, int n, int h, int64_t fa, int64_t total,
                         hipStream_t hs) {
  hipError_t e = hipSuccess;
  if (!m->side) e = hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking);
  if (e == hipSuccess && !m->fork_ev) e = hipEventCreateWithFlags(&m->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess && !m->join_ev) e = hipEventCreateWithFlags(&m->join_ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  // fork: the second half on the side stream; join before the caller's next
  // work.  The two halves' launches are issued alternately, so that the
  // second half can start at once even when the host issues a step just
  // before the device runs it.
  e = hipEventRecord(m->fork_ev, hs);
  if (e == hipSuccess) e = hipStreamWaitEvent(m->side, m->fork_ev, 0);
  const WsView w = model_ws(m);
  const LaunchSet la = launch_set(dev, h, fa, hs, 0, w);
  const LaunchSet lb = launch_set(dev + split_desc_offset(h, fa, m->plan.input_multiple), n - h, total - fa, m->side, fa,
                                  w);
  if (e == hipSuccess) e = launch_pack(m, la);
  if (e == hipSuccess) e = launch_pack(m, lb);
  for (size_t oi = 0; e == hipSuccess && oi < m->plan.ops.size(); ++oi) {
    e = launch_op(m, oi, la);
    if (e == hipSuccess) e = launch_op(m, oi, lb);
  }
  if (e == hipSuccess) e = hipEventRecord(m->join_ev, m->side);
  if (e == hipSuccess) e = hipStreamWaitEvent(hs, m->join_ev, 0);
  return e;
}

void commit_step(int n, sc_stream* const* streams, const int32_t* n_frames) {
  for (int i = 0; i < n; ++i) {
    streams[i]->pos += n_frames[i];
    streams[i]->parity ^= 1;
  }
}

}  // namespace sc

namespace {

// Captures the step graph for the current workspace if it is missing or
// stale.  Its descriptor buffer is reallocated only with the device idle (the
// workspace has just grown, or the graph was just enabled).
sc_status ensure_graph(sc_model* m) {
  if (m->graph_exec && m->graph_frames == m->ws_cap) return SC_OK;
  hipError_t e;
  if (m->graph_exec) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipGraphExecDestroy(m->graph_exec);
    m->graph_exec = nullptr;
  }
  const size_t bytes = desc_bytes(m->graph_streams, m->ws_cap, m->plan.input_multiple);
  if (m->graph_desc_bytes < bytes) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipFree(m->graph_desc);
    m->graph_desc = nullptr;
    m->graph_desc_bytes = 0;
    e = hipMalloc(reinterpret_cast<void**>(&m->graph_desc), bytes);
    if (e != hipSuccess) return fail(SC_ENOMEM, "step graph descriptor allocation failed");
    m->graph_desc_bytes = bytes;
  }
  if (!m->capture_stream) {
    e = hipStreamCreateWithFlags(&m->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  }
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(m->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const hipError_t le = enqueue_kernels(m, m->graph_desc, m->graph_streams, m->ws_cap, m->capture_stream);
  e = hipStreamEndCapture(m->capture_stream, &g);
  if (le != hipSuccess) { if (g) hipGraphDestroy(g); return hip_fail(le, "step capture"); }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&m->graph_exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) { m->graph_exec = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
  m->graph_frames = m->ws_cap;
  return SC_OK;
}

sc_status run_step(sc_model* m, int n, sc_stream* const* streams, const float* const* d_in,
                   const int32_t* n_frames, float* const* d_out, hipStream_t hs) {
  int64_t total = 0;
  sc_status st = validate_step(m, n, streams, d_in, n_frames, d_out, &total);
  if (st != SC_OK) return st;
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  st = ensure_workspace(m, total);
  if (st != SC_OK) return st;
  if (m->prof_on && m->prof_used > 0) {
    // fold the previous step's launch timings, so that one step's worth of
    // events is reused (the host waits for that step: profiling only)
    e = prof_fold(m);
    if (e != hipSuccess) return hip_fail(e, "profile fold");
  }

  // the step graph serves steps of up to graph_streams streams (and any size
  // up to the workspace); timed or calibrating steps launch one by one
  const bool graph = m->graph_streams >= n && !m->prof_on && !m->amax_on;
  const int cap = graph ? m->graph_streams : n;
  int64_t fa = 0;
  const int h = (graph || m->prof_on || m->amax_on) ? 0 : choose_split(m, n, n_frames, total, &fa);

  // ---- descriptors ----
  DescSlot& slot = m->ring[m->ring_next];
  m->ring_next = (m->ring_next + 1) % kRing;
  if (slot.pending) {
    e = hipEventSynchronize(slot.done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    slot.pending = false;
  }
  // a split step's two descriptors sit one after the other in the slot
  const int64_t gr = m->plan.input_multiple;
  const size_t off_b = h ? split_desc_offset(h, fa, gr) : 0;
  const size_t need = h ? off_b + desc_bytes(n - h, total - fa, gr) : desc_bytes(cap, total, gr);
  if (slot.cap < need) {
    if (slot.host) hipHostFree(slot.host);
    if (slot.dev) hipFree(slot.dev);
    slot.host = nullptr;
    slot.host_dev = nullptr;
    slot.dev = nullptr;
    const size_t cap = std::max<size_t>(need * 2, 64 * 1024);
    // coherent: the upload kernel reads the host's latest writes, never a
    // cached copy of this slot's previous use
    void* hd = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&slot.host), cap, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer(&hd, slot.host, 0) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&slot.dev), cap) != hipSuccess) {
      slot.cap = 0;
      return fail(SC_ENOMEM, "descriptor allocation failed");
    }
    slot.host_dev = static_cast<const unsigned char*>(hd);
    slot.cap = cap;
  }
  if (!slot.done) {
    e = hipEventCreateWithFlags(&slot.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  }
  if (h) {
    fill_descriptor(slot.host, h, h, streams, d_in, n_frames, d_out, fa, gr);
    fill_descriptor(slot.host + off_b, n - h, n - h, streams + h, d_in + h, n_frames + h, d_out + h, total - fa, gr);
  } else {
    fill_descriptor(slot.host, n, cap, streams, d_in, n_frames, d_out, total, gr);
  }
  if (graph) {
    st = ensure_graph(m);
    if (st != SC_OK) return st;
  }
  if (m->has_last) {
    e = hipStreamWaitEvent(hs, m->last_done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  // a kernel reads the descriptor over PCIe: one short launch instead of a DMA
  // copy and its engine hand-off before the step's first kernel
  // (the frame table's spare slots at the end are never used: not copied)
  e = launch_upload(slot.host_dev, graph ? m->graph_desc : slot.dev, need - kFentPad * sizeof(int32_t), hs);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  if (h) {
    e = enqueue_split(m, slot.dev, n, h, fa, total, hs);
  } else {
    e = graph ? hipGraphLaunch(m->graph_exec, hs) : enqueue_kernels(m, slot.dev, n, total, hs);
  }
  if (e == hipSuccess) e = hipEventRecord(slot.done, hs);
  if (e != hipSuccess) {
    for (int i = 0; i < n; ++i) streams[i]->bad = true;
    // a half already on the side stream must not outlive the failed step
    // (nothing later orders against it)
    if (h && m->side) hipStreamSynchronize(m->side);
    return hip_fail(e, "kernel launch");
  }
  slot.pending = true;
  m->last_done = slot.done;   // one event per step: the slot's also orders later work
  m->has_last = true;
  commit_step(n, streams, n_frames);
  return SC_OK;
}

}  // namespace


sc_status sc::run_step_locked(sc_model* m, int n, sc_stream* const* streams, const float* const* d_in,
                              const int32_t* n_frames, float* const* d_out, hipStream_t hs) {
  return run_step(m, n, streams, d_in, n_frames, d_out, hs);
}

sc_status sc::fail_hip(hipError_t e, const char* what) { return hip_fail(e, what); }

namespace {

void fill_info(const Plan& p, sc_model_info* out) {
  std::memset(out, 0, sizeof(*out));
  out->in_channels = p.in_channels;
  out->out_channels = p.out_channels;
  out->out_num = (int32_t)p.out_rate.num;
  out->out_den = (int32_t)p.out_rate.den;
  out->input_multiple = p.input_multiple;
  out->n_launch = (int32_t)p.ops.size();
  out->latency = p.latency;
  out->warmup = p.warmup;
  out->state_bytes_per_stream = p.state_floats * (int64_t)sizeof(float);
  out->state_alloc_per_stream = std::max<int64_t>(p.state_alloc_floats, 1) * (int64_t)sizeof(float);
}

sc_status zero_state(sc_stream* s, hipStream_t hs) {
  sc_model* m = s->m;
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (m->has_last) {
    e = hipStreamWaitEvent(hs, m->last_done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  e = launch_fill_zero(s->d_state, std::max<int64_t>(m->plan.state_alloc_floats, 1), hs);
  if (e == hipSuccess) e = hipEventRecord(m->own_done, hs);
  if (e != hipSuccess) return hip_fail(e, "state reset");
  m->last_done = m->own_done;
  m->has_last = true;
  s->pos = 0;
  s->parity = 0;
  s->bad = false;
  return SC_OK;
}

}  // namespace

extern "C" {

const char* sc_last_error(void) { return last_error_cstr(); }

sc_status sc_plan(const sc_node* nodes, int32_t n_nodes, sc_model_info* out) {
  if (!out) return fail(SC_EINVAL, "null output");
  Plan p;
  std::string err;
  sc_status st = build_plan(nodes, n_nodes, 0, p, err);
  if (st != SC_OK) return fail(st, err);
  fill_info(p, out);
  return SC_OK;
}

}  // extern "C"

namespace {

// sc_model_create / sc_model_create_mixed: `precision` for every layer, or
// one precision per layer (`layer_prec`, node order) when it is not null.
sc_status create_model(const sc_node* nodes, int32_t n_nodes, const float* weights, size_t n_weights,
                       sc_precision precision, const int32_t* layer_prec, const float* act_scales,
                       uint32_t options, int32_t device, sc_model** out) {
  if (!out) return fail(SC_EINVAL, "null output");
  *out = nullptr;
  auto known = [](int32_t p) { return p == SC_FP32 || p == SC_BF16 || p == SC_FP8E4M3; };
  if (!layer_prec && !known(precision)) return fail(SC_EINVAL, "unknown precision");
  sc_model* m = new (std::nothrow) sc_model();
  if (!m) return fail(SC_ENOMEM, "host allocation failed");
  std::string err;
  sc_status st = build_plan(nodes, n_nodes, options, m->plan, err);
  if (st != SC_OK) { delete m; return fail(st, err); }
  const int n_layers = (int)m->plan.layer_node.size();
  auto prec_id_of = [](int32_t p) { return p == SC_FP32 ? 0 : (p == SC_BF16 ? 1 : 2); };
  m->layer_prec.assign(n_layers, prec_id_of(precision));
  if (layer_prec) {
    int lowest = 0;
    for (int i = 0; i < n_layers; ++i) {
      if (!known(layer_prec[i])) { delete m; return fail(SC_EINVAL, "unknown precision in layer_precision"); }
      m->layer_prec[i] = prec_id_of(layer_prec[i]);
      lowest = std::max(lowest, m->layer_prec[i]);
    }
    precision = lowest == 0 ? SC_FP32 : (lowest == 1 ? SC_BF16 : SC_FP8E4M3);
  }
  if ((options & SC_MODEL_NO_MFMA) && precision != SC_FP32) {
    delete m;
    return fail(SC_EINVAL, "SC_MODEL_NO_MFMA needs SC_FP32");
  }
  if (!weights || (int64_t)n_weights != m->plan.n_weights) {
    delete m;
    return fail(SC_EINVAL, "weights missing or of the wrong length (expected " +
                               std::to_string(m->plan.n_weights) + ")");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    delete m;
    return fail(SC_EDEVICE, "no such HIP device");
  }
  m->device = device;
  m->prec = precision;
  m->options = options;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->own_done, hipEventDisableTiming);
  // the no-alloc path's scratch array on this device (once per device)
  if (e == hipSuccess) e = scratch_setup(device);
  if (e != hipSuccess) { delete m; return hip_fail(e, "device setup"); }
  if (act_scales) {
    m->act_scales.assign(act_scales, act_scales + n_layers);
    m->have_scales = true;
  } else {
    m->act_scales.assign(n_layers, 1.0f);
  }
  m->opdev.resize(m->plan.ops.size());
  for (size_t i = 0; i < m->plan.ops.size(); ++i) {
    Op& op = m->plan.ops[i];
    OpDev& od = m->opdev[i];
    if (op.kind == K_DELAY_ADD) continue;
    const float* w = weights + op.w_off;
    const float* b = weights + op.b_off;
    const int prec_id = op.layer >= 0 ? m->layer_prec[op.layer] : 0;
    bool mfma = false, fp32_input = false;
    if (!(options & SC_MODEL_NO_MFMA) && op.in_buf >= 0 && op.out_buf >= 0) {
      // (a fused skip reads the window at the output rate: stride-1 convs only)
      if (op.kind == K_CONV) mfma = conv_mfma_supported(op.cin, op.cout, op.k, op.stride, prec_id) &&
                                    (op.stride == 1 || !op.residual);
      else mfma = convt_mfma_supported(op.cin, op.cout, op.stride, prec_id);
      // a narrow layer reading the model input (the latents) runs on FP32
      // MFMA in every precision: its input is never rounded
      if (!mfma && op.kind == K_CONV && op.in_buf == m->plan.input_buf &&
          conv_mfma_fp32_input_supported(op.cin, op.cout, op.k, op.stride))
        mfma = fp32_input = true;
    }
    op.impl = mfma ? IMPL_MFMA : IMPL_VALU;
    op.no_twin = fp32_input ? 1 : 0;
    od.prec = (mfma && !fp32_input) ? prec_id : 0;
    op.prec = od.prec;
    if (od.prec == 2) m->any_fp8 = true;
    if (mfma && op.kind == K_CONV && !(options & SC_MODEL_NO_WIN)) {
      const int64_t min_frames = op.in_rate.of(m->plan.input_multiple);
      od.win_rows = conv_win_rows(op.cin, op.cout, op.k, op.dil, op.stride, op.cache_len, min_frames, prec_id);
      if (od.win_rows > 0) op.impl = IMPL_WIN;
    }
    if (mfma) {
      std::vector<uint8_t> packed;
      std::vector<float> wscale;
      if (op.kind == K_CONV) pack_conv_mfma(w, op.cout, op.cin, op.k, od.prec, packed, wscale);
      else pack_convt_mfma(w, op.cin, op.cout, op.stride, od.prec, packed, wscale);
      e = upload(reinterpret_cast<uint8_t**>(&od.W), packed.data(), packed.size());
      if (e == hipSuccess && !wscale.empty()) e = upload(&od.wscale, wscale.data(), wscale.size());
      m->weight_bytes += (int64_t)packed.size() + (int64_t)wscale.size() * 4;
    } else {
      std::vector<float> packed = op.kind == K_CONV ? pack_conv_valu(w, op.cout, op.cin, op.k)
                                                    : pack_convt_valu(w, op.cin, op.cout, op.stride);
      e = upload(reinterpret_cast<float**>(&od.W), packed.data(), packed.size());
      m->weight_bytes += (int64_t)packed.size() * 4;
    }
    if (e == hipSuccess) e = upload(&od.B, b, (size_t)op.cout);
    m->weight_bytes += (int64_t)op.cout * 4;
    if (e != hipSuccess) { free_model(m); return hip_fail(e, "weight upload"); }
  }
  if (!(options & SC_MODEL_NO_OUT_FUSION)) fuse_output_convs(m->plan);
  finalize_plan(m->plan, !(options & SC_MODEL_NO_TWIN));
  if (!(options & SC_MODEL_NO_CONVT_FUSION)) fuse_convt_windows(m);
  if (!(options & SC_MODEL_NO_INPUT_DIRECT)) mark_input_direct(m);
  if (!(options & SC_MODEL_NO_PAIR_FUSION)) fuse_conv_pairs(m);
  e = hipMalloc(reinterpret_cast<void**>(&m->d_amax), std::max(n_layers, 1) * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->d_amax, 0, std::max(n_layers, 1) * sizeof(float));
  if (e != hipSuccess) { free_model(m); return hip_fail(e, "amax buffer"); }
  *out = m;
  return SC_OK;
}

}  // namespace

extern "C" {

sc_status sc_model_create(const sc_node* nodes, int32_t n_nodes, const float* weights, size_t n_weights,
                          sc_precision precision, const float* act_scales, uint32_t options, int32_t device,
                          sc_model** out) {
  return create_model(nodes, n_nodes, weights, n_weights, precision, nullptr, act_scales, options, device, out);
}

sc_status sc_model_create_mixed(const sc_node* nodes, int32_t n_nodes, const float* weights, size_t n_weights,
                                const int32_t* layer_precision, const float* act_scales, uint32_t options,
                                int32_t device, sc_model** out) {
  if (!layer_precision) return fail(SC_EINVAL, "null layer_precision");
  return create_model(nodes, n_nodes, weights, n_weights, SC_FP32, layer_precision, act_scales, options, device,
                      out);
}

sc_status sc_model_info_get(const sc_model* m, sc_model_info* out) {
  if (!m || !out) return fail(SC_EINVAL, "null argument");
  fill_info(m->plan, out);
  out->weight_bytes = m->weight_bytes;
  int n_mfma = 0;
  (void)n_mfma;
  return SC_OK;
}

int32_t sc_model_n_layers(const sc_model* m) { return m ? (int32_t)m->plan.layer_node.size() : -1; }

sc_status sc_model_enable_graph(sc_model* m, int32_t max_streams) {
  if (!m || max_streams < 0) return fail(SC_EINVAL, "null model or negative stream count");
  std::lock_guard<std::mutex> g(m->mu);
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (m->graph_exec) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipGraphExecDestroy(m->graph_exec);
    m->graph_exec = nullptr;
  }
  m->graph_streams = max_streams;
  return SC_OK;
}

sc_status sc_model_reserve(sc_model* m, int64_t max_step_frames) {
  if (!m || max_step_frames < 1 || max_step_frames > INT32_MAX / 4)
    return fail(SC_EINVAL, "null model or step size out of range");
  std::lock_guard<std::mutex> g(m->mu);
  const hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return ensure_workspace(m, max_step_frames);
}

sc_status sc_model_set_act_scales(sc_model* m, const float* s) {
  if (!m || !s) return fail(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(m->mu);
  const int n = (int)m->plan.layer_node.size();
  for (int i = 0; i < n; ++i)
    if (!(s[i] > 0.f) || !std::isfinite(s[i])) return fail(SC_EINVAL, "activation scales must be positive and finite");
  if (m->ws_pins > 0)
    return fail(SC_ESTATE, "a server's captured step graphs hold this model's scales; destroy it first");
  if (m->graph_exec) {   // the captured launches hold the old scales
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    hipGraphExecDestroy(m->graph_exec);
    m->graph_exec = nullptr;
  }
  m->act_scales.assign(s, s + n);
  m->have_scales = true;
  return SC_OK;
}

sc_status sc_model_enable_amax(sc_model* m, int32_t enable) {
  if (!m) return fail(SC_EINVAL, "null model");
  std::lock_guard<std::mutex> g(m->mu);
  if (enable && m->n_pairs > 0)
    return fail(SC_EINVAL, "activation maxima need every layer's input: calibrate on an FP32 model (or one created "
                           "with SC_MODEL_NO_PAIR_FUSION)");
  m->amax_on = enable != 0;
  return SC_OK;
}

sc_status sc_model_read_amax(sc_model* m, float* out, int32_t reset) {
  if (!m || !out) return fail(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(m->mu);
  const int n = (int)m->plan.layer_node.size();
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && n > 0) e = hipMemcpy(out, m->d_amax, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && reset && n > 0) e = hipMemset(m->d_amax, 0, n * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "amax readback");
  return SC_OK;
}

sc_status sc_model_calibrated_scales(sc_model* m, float* out) {
  if (!m || !out) return fail(SC_EINVAL, "null argument");
  const sc_status st = sc_model_read_amax(m, out, 0);
  if (st != SC_OK) return st;
  // static activation scale of a layer: the largest |activated input| seen
  // while calibrating, with a 25% margin against unseen peaks
  constexpr float kMargin = 1.25f, kFloor = 1e-6f;
  const int n = (int)m->plan.layer_node.size();
  for (int i = 0; i < n; ++i) out[i] = std::max(out[i] * kMargin, kFloor);
  return SC_OK;
}

namespace {
// Drops one reference; frees the model when none is left.
void model_unref(sc_model* m) {
  bool last;
  {
    std::lock_guard<std::mutex> g(m->mu);
    last = --m->refs == 0;
  }
  if (last) free_model(m);
}
}  // namespace

void sc_model_destroy(sc_model* m) {
  if (m) model_unref(m);
}

sc_status sc_model_profile(sc_model* m, int32_t enable) {
  if (!m) return fail(SC_EINVAL, "null model");
  std::lock_guard<std::mutex> g(m->mu);
  hipSetDevice(m->device);
  hipError_t e = prof_fold(m);
  if (e != hipSuccess) return hip_fail(e, "profile fold");
  m->prof_on = enable != 0;
  if (m->prof_on) {
    m->prof.assign(m->plan.ops.size(), sc_op_profile{});
    for (size_t i = 0; i < m->plan.ops.size(); ++i) {
      const Op& op = m->plan.ops[i];
      sc_op_profile& p = m->prof[i];
      p.kind = op.kind;
      p.impl = op.impl;
      p.precision = m->opdev[i].prec;
      p.node = op.node;
      p.cin = op.cin; p.cout = op.cout; p.k = op.k; p.dilation = op.dil; p.stride = op.stride;
      p.cache_len = op.cache_len; p.residual = op.residual; p.a0 = op.A0; p.a1 = op.A1;
      p.rate_in_num = (int32_t)op.in_rate.num; p.rate_in_den = (int32_t)op.in_rate.den;
      p.rate_out_num = (int32_t)op.out_rate.num; p.rate_out_den = (int32_t)op.out_rate.den;
    }
  }
  return SC_OK;
}

sc_status sc_model_profile_read(sc_model* m, sc_op_profile* out, int32_t max_ops, int32_t* n_ops) {
  if (!m || !n_ops) return fail(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(m->mu);
  hipSetDevice(m->device);
  hipError_t e = prof_fold(m);
  if (e != hipSuccess) return hip_fail(e, "profile fold");
  *n_ops = (int32_t)m->plan.ops.size();
  for (int i = 0; out && i < max_ops && i < (int)m->prof.size(); ++i) out[i] = m->prof[i];
  return SC_OK;
}

sc_status stream_create(sc_model* m, int32_t max_frames, uint32_t flags, void* hip_stream, sc_stream** out) {
  if (!m || !out) return fail(SC_EINVAL, "null argument");
  *out = nullptr;
  if (max_frames < 1 || max_frames % m->plan.input_multiple != 0)
    return fail(SC_ELENGTH, "max_buffer_frames must be >= 1 and a multiple of the total stride");
  if (flags & ~(uint32_t)SC_FLAG_WARMUP_MASK) return fail(SC_EINVAL, "unknown flags");
  std::lock_guard<std::mutex> g(m->mu);
  hipError_t e = hipSetDevice(m->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  sc_stream* s = new (std::nothrow) sc_stream();
  if (!s) return fail(SC_ENOMEM, "host allocation failed");
  s->m = m;
  s->max_frames = max_frames;
  s->flags = flags;
  const size_t bytes = (size_t)std::max<int64_t>(m->plan.state_alloc_floats, 1) * sizeof(float);
  e = hipMalloc(reinterpret_cast<void**>(&s->d_state), bytes);
  if (e != hipSuccess) { delete s; return fail(SC_ENOMEM, "state allocation failed"); }
  sc_status st = zero_state(s, static_cast<hipStream_t>(hip_stream));
  if (st != SC_OK) { hipFree(s->d_state); delete s; return st; }
  m->refs++;
  *out = s;
  return SC_OK;
}

namespace {
// Exported state: header, then the device state allocation (both copies).
struct StateHeader {
  uint32_t magic;             // 'SCST'
  uint32_t version;
  int64_t state_alloc_floats;
  int64_t latency, warmup;
  int32_t precision, n_ops;
  int32_t in_channels, out_channels;
  int64_t pos;
  int32_t parity, reserved;
  uint64_t op_prec_sig;       // per-op operand precisions (the twin cache layout depends on them)
};
constexpr uint32_t kStateMagic = 0x54534353u;   // "SCST" little-endian

StateHeader state_header(const sc_model* m) {
  StateHeader h{};
  h.magic = kStateMagic;
  h.version = 2;
  h.state_alloc_floats = std::max<int64_t>(m->plan.state_alloc_floats, 1);
  h.latency = m->plan.latency;
  h.warmup = m->plan.warmup;
  h.precision = (int32_t)m->prec;
  h.n_ops = (int32_t)m->plan.ops.size();
  h.in_channels = m->plan.in_channels;
  h.out_channels = m->plan.out_channels;
  uint64_t sig = 1469598103934665603ull;   // FNV-1a over the ops' precisions
  for (const Op& op : m->plan.ops) sig = (sig ^ (uint64_t)(op.prec + 1)) * 1099511628211ull;
  h.op_prec_sig = sig;
  return h;
}
}  // namespace

int64_t sc_stream_state_bytes(const sc_model* m) {
  if (!m) return -1;
  return (int64_t)sizeof(StateHeader) + std::max<int64_t>(m->plan.state_alloc_floats, 1) * (int64_t)sizeof(float);
}

sc_status stream_export(sc_stream* s, void* host, int64_t bytes) {
  if (!s || !host) return fail(SC_EINVAL, "null argument");
  sc_model* m = s->m;
  if (bytes < sc_stream_state_bytes(m)) return fail(SC_EINVAL, "buffer smaller than sc_stream_state_bytes");
  std::lock_guard<std::mutex> g(m->mu);
  if (s->bad) return fail(SC_ESTATE, "stream saw a device error; call stream_reset");
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess && m->has_last) e = hipEventSynchronize(m->last_done);
  StateHeader h = state_header(m);
  h.pos = s->pos;
  h.parity = s->parity;
  std::memcpy(host, &h, sizeof(h));
  if (e == hipSuccess)
    e = hipMemcpy(static_cast<unsigned char*>(host) + sizeof(h), s->d_state,
                  (size_t)h.state_alloc_floats * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "state export");
  return SC_OK;
}

sc_status stream_import(sc_stream* s, const void* host, int64_t bytes) {
  if (!s || !host) return fail(SC_EINVAL, "null argument");
  sc_model* m = s->m;
  if (bytes != sc_stream_state_bytes(m)) return fail(SC_EINVAL, "size differs from sc_stream_state_bytes");
  StateHeader h;
  std::memcpy(&h, host, sizeof(h));
  StateHeader want = state_header(m);
  if (h.magic != want.magic || h.version != want.version || h.state_alloc_floats != want.state_alloc_floats ||
      h.latency != want.latency || h.warmup != want.warmup || h.precision != want.precision ||
      h.n_ops != want.n_ops || h.in_channels != want.in_channels || h.out_channels != want.out_channels ||
      h.op_prec_sig != want.op_prec_sig ||
      h.pos < 0 || (h.parity != 0 && h.parity != 1))
    return fail(SC_EINVAL, "state of another graph or precision");
  std::lock_guard<std::mutex> g(m->mu);
  hipError_t e = hipSetDevice(m->device);
  if (e == hipSuccess && m->has_last) e = hipEventSynchronize(m->last_done);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_state, static_cast<const unsigned char*>(host) + sizeof(h),
                  (size_t)h.state_alloc_floats * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    s->bad = true;
    return hip_fail(e, "state import");
  }
  s->pos = h.pos;
  s->parity = h.parity;
  s->bad = false;
  return SC_OK;
}

sc_status stream_process(sc_stream* s, const float* d_in, int32_t n_frames, float* d_out, void* hip_stream) {
  if (!s) return fail(SC_EINVAL, "null stream");
  std::lock_guard<std::mutex> g(s->m->mu);
  return run_step(s->m, 1, &s, &d_in, &n_frames, &d_out, static_cast<hipStream_t>(hip_stream));
}

sc_status sc_process_batch(sc_model* m, int32_t n, sc_stream* const* streams, const float* const* d_in,
                           const int32_t* n_frames, float* const* d_out, void* hip_stream) {
  if (!m) return fail(SC_EINVAL, "null model");
  std::lock_guard<std::mutex> g(m->mu);
  return run_step(m, n, streams, d_in, n_frames, d_out, static_cast<hipStream_t>(hip_stream));
}

sc_status stream_reset(sc_stream* s, void* hip_stream) {
  if (!s) return fail(SC_EINVAL, "null stream");
  std::lock_guard<std::mutex> g(s->m->mu);
  return zero_state(s, static_cast<hipStream_t>(hip_stream));
}

int64_t stream_position(const sc_stream* s) { return s ? s->pos : -1; }

void stream_destroy(sc_stream* s) {
  if (!s) return;
  sc_model* m = s->m;
  {
    std::lock_guard<std::mutex> g(m->mu);
    hipSetDevice(m->device);
    if (m->has_last) hipEventSynchronize(m->last_done);
    hipFree(s->d_state);
  }
  delete s;
  model_unref(m);
}

}  // extern "C"
