// Serving loop: continuous batching of many live streams on one model.
//
// A worker thread forms one batched step at a time from the streams' queued
// buffers, enqueues it on the server's HIP stream through a ring of step
// contexts (pinned host staging, device staging, descriptor, event and --
// with use_graph -- one captured hipGraph of the step's kernels, sized for the
// largest step and replayed for any smaller one), and finalizes completed
// contexts: outputs are copied to the buffers' tickets and their latency is
// stamped.  Up to kCtx steps are in flight, so the next step is formed while
// the device runs the previous one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "model_internal.h"

using namespace sc;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kCtx = 3;
constexpr size_t kSplitSlack = 512;   // a split step's second descriptor starts 256-byte aligned

struct Ticket {
  int64_t id = 0;
  int64_t stream_id = 0;
  int32_t frames = 0;
  std::vector<float> in;    // [C_in][frames]
  std::vector<float> out;   // [C_out][frames * rate]
  Clock::time_point t_submit, t_done;
  bool done = false;
  bool failed = false;      // its step could not be enqueued
  bool discard = false;     // SC_SUBMIT_DISCARD
};

struct SStream {
  int64_t id = 0;
  sc_stream* s = nullptr;
  std::deque<Ticket*> queue;
  bool admitted = false;
  bool closing = false;
  int inflight = 0;
};

struct Part {               // one stream's share of a step
  SStream* st;
  std::vector<Ticket*> tickets;
  int32_t frames = 0;
  int64_t in_off = 0, out_off = 0;   // floats into the staging buffers
};

struct StepCtx {
  unsigned char* desc_host = nullptr;
  const unsigned char* desc_hdev = nullptr;   // device address of desc_host
  unsigned char* desc_dev = nullptr;
  float* in_host = nullptr;
  const float* in_hdev = nullptr;             // device address of in_host
  float* in_dev = nullptr;
  float* out_host = nullptr;
  float* out_dev = nullptr;
  hipEvent_t done = nullptr;
  hipGraphExec_t exec = nullptr;
  bool busy = false;
  std::vector<Part> parts;
  int64_t out_floats = 0;
};

}  // namespace

struct sc_server {
  sc_model* m = nullptr;
  sc_server_config cfg{};
  hipStream_t hs = nullptr;
  int32_t cin = 0, cout = 0;
  int64_t out_num = 1, out_den = 1;
  int64_t max_frames = 0;      // input frames of the largest step
  int max_admit = 0;
  int64_t fixed_bytes = 0, per_stream_bytes = 0;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::map<int64_t, std::unique_ptr<SStream>> streams;  // open streams by id
  std::deque<SStream*> waiting;                          // admission FIFO
  std::unordered_map<int64_t, std::unique_ptr<Ticket>> tickets;
  int64_t next_ticket = 1;
  int admitted = 0;
  int queued = 0;              // buffers submitted and not yet finalized
  StepCtx ctx[kCtx];
  int next_ctx = 0;
  std::thread worker;
  bool stop = false;
  std::string worker_error;
  sc_server_stats stats{};
  std::deque<std::pair<int64_t, double>> lat_log;   // (ticket, latency) of discarded buffers
};

namespace {

sc_status srv_fail(sc_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

int64_t out_frames_of(const sc_server* s, int64_t frames) { return frames * s->out_num / s->out_den; }

void free_ctx(StepCtx& c) {
  if (c.exec) hipGraphExecDestroy(c.exec);
  if (c.done) hipEventDestroy(c.done);
  if (c.desc_host) hipHostFree(c.desc_host);
  if (c.in_host) hipHostFree(c.in_host);
  if (c.out_host) hipHostFree(c.out_host);
  hipFree(c.desc_dev);
  hipFree(c.in_dev);
  hipFree(c.out_dev);
  c = StepCtx();
}

// Copies a finished context's outputs to its tickets and releases streams
// whose last buffer it held.  Called with srv->mu held.
void finalize(sc_server* srv, StepCtx& c, bool failed = false) {
  const auto now = Clock::now();
  for (Part& p : c.parts) {
    int64_t t_off = 0;
    const int64_t T = out_frames_of(srv, p.frames);
    for (Ticket* t : p.tickets) {
      const int64_t Tt = out_frames_of(srv, t->frames);
      srv->queued--;
      if (t->discard) {
        if (!failed)
          srv->lat_log.emplace_back(t->id, std::chrono::duration<double>(now - t->t_submit).count());
        t_off += Tt;
        srv->tickets.erase(t->id);
        continue;
      }
      t->out.resize((size_t)srv->cout * Tt);
      for (int co = 0; co < srv->cout; ++co)
        std::memcpy(&t->out[(size_t)co * Tt], c.out_host + p.out_off + (int64_t)co * T + t_off, Tt * sizeof(float));
      t_off += Tt;
      t->t_done = now;
      t->done = true;
      t->failed = failed;
    }
    SStream* st = p.st;
    st->inflight--;
    if (st->closing && st->queue.empty() && st->inflight == 0) {
      stream_destroy(st->s);
      st->s = nullptr;
      srv->admitted--;
      srv->streams.erase(st->id);
    }
  }
  c.parts.clear();
  c.busy = false;
  srv->cv_done.notify_all();
}

// Fails every queued buffer of a stream whose state is broken (a step that
// included it could not be enqueued).  Called with srv->mu held.
void fail_queued(sc_server* srv, SStream* st) {
  const auto now = Clock::now();
  while (!st->queue.empty()) {
    Ticket* t = st->queue.front();
    st->queue.pop_front();
    srv->queued--;
    if (t->discard) {
      srv->tickets.erase(t->id);
      continue;
    }
    t->t_done = now;
    t->done = true;
    t->failed = true;
  }
  srv->cv_done.notify_all();
}

// Captures the context's step kernels, sized for the largest step.  Done at
// server creation on the creating thread (a capture on the worker thread could
// be invalidated by device-wide calls, such as a free, from other threads).
// Called with the model's lock held.
hipError_t capture_step(sc_server* srv, StepCtx& c) {
  sc_model* m = srv->m;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(srv->hs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const bool prof = m->prof_on, amax = m->amax_on;
  m->prof_on = false;
  m->amax_on = false;
  const hipError_t le = enqueue_kernels(m, c.desc_dev, srv->cfg.max_streams, srv->max_frames, srv->hs);
  m->prof_on = prof;
  m->amax_on = amax;
  e = hipStreamEndCapture(srv->hs, &g);
  if (le != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return le;
  }
  if (e != hipSuccess) return e;
  e = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) c.exec = nullptr;
  return e;
}

// Launches the context's step kernels (its captured graph, or one by one).
hipError_t launch_step(sc_server* srv, StepCtx& c, int n, int64_t total) {
  sc_model* m = srv->m;
  if (!srv->cfg.use_graph) return enqueue_kernels(m, c.desc_dev, n, total, srv->hs);
  if (!c.exec) return hipErrorInvalidValue;   // captured at creation
  return hipGraphLaunch(c.exec, srv->hs);
}

void worker_main(sc_server* srv) {
  hipSetDevice(srv->m->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    // admission, first come first served
    while (!srv->waiting.empty() && srv->admitted < srv->max_admit) {
      SStream* st = srv->waiting.front();
      srv->waiting.pop_front();
      sc_stream* s = nullptr;
      const sc_status rc = stream_create(srv->m, srv->cfg.max_buffer_frames, srv->cfg.stream_flags, srv->hs, &s);
      if (rc != SC_OK) {
        srv->worker_error = std::string("stream_create: ") + sc_last_error();
        srv->waiting.push_front(st);
        break;
      }
      st->s = s;
      st->admitted = true;
      srv->admitted++;
    }
    // finalize finished contexts
    for (auto& c : srv->ctx)
      if (c.busy && hipEventQuery(c.done) == hipSuccess) finalize(srv, c);
    bool work = false;
    for (auto& kv : srv->streams) work |= kv.second->admitted && !kv.second->queue.empty();
    if (work) {
      // a failed step left these streams' state behind their buffers: their
      // queued buffers fail rather than continue a broken stream
      std::vector<int64_t> gone;
      for (auto& kv : srv->streams) {
        SStream* st = kv.second.get();
        if (!st->admitted || !st->s || !st->s->bad || st->queue.empty()) continue;
        fail_queued(srv, st);
        if (st->closing && st->inflight == 0) gone.push_back(st->id);
      }
      for (int64_t id : gone) {
        stream_destroy(srv->streams[id]->s);
        srv->admitted--;
        srv->streams.erase(id);
      }
      work = false;
      for (auto& kv : srv->streams) work |= kv.second->admitted && !kv.second->queue.empty();
      if (!work) continue;
    }
    if (!work) {
      bool any_busy = false;
      for (auto& c : srv->ctx) any_busy |= c.busy;
      if (srv->stop && !any_busy && srv->queued == 0) break;
      if (any_busy) {
        // wait for the oldest step outside the lock, then finalize it
        StepCtx* oldest = nullptr;
        for (int i = 0; i < kCtx; ++i) {
          StepCtx& c = srv->ctx[(srv->next_ctx + i) % kCtx];
          if (c.busy) { oldest = &c; break; }
        }
        lk.unlock();
        hipEventSynchronize(oldest->done);
        lk.lock();
        finalize(srv, *oldest);
      } else {
        srv->cv.wait_for(lk, std::chrono::milliseconds(2));
      }
      continue;
    }
    StepCtx& c = srv->ctx[srv->next_ctx];
    if (c.busy) {
      // the ring is full: retire its oldest step first (this may free slots)
      lk.unlock();
      hipEventSynchronize(c.done);
      lk.lock();
      finalize(srv, c);
      continue;
    }
    srv->next_ctx = (srv->next_ctx + 1) % kCtx;
    // the next step: one buffer per admitted stream, merging queued buffers.
    // A stream counts the step as in flight from here on, so that closing it
    // cannot free it while the step is formed or running.
    std::vector<Part> parts;
    int64_t total = 0;
    for (auto& kv : srv->streams) {
      SStream* st = kv.second.get();
      if (!st->admitted || st->queue.empty()) continue;
      if (st->s->bad) continue;   // (its buffers were failed above)
      Part p;
      p.st = st;
      while (!st->queue.empty() && p.frames + st->queue.front()->frames <= srv->cfg.max_buffer_frames) {
        p.frames += st->queue.front()->frames;
        p.tickets.push_back(st->queue.front());
        st->queue.pop_front();
      }
      st->inflight++;
      total += p.frames;
      parts.push_back(std::move(p));
      if ((int)parts.size() == srv->cfg.max_streams) break;
    }
    // stage inputs (channel-major per stream, merged buffers back to back)
    const int n = (int)parts.size();
    std::vector<sc_stream*> ss(n);
    std::vector<const float*> din(n);
    std::vector<float*> dout(n);
    std::vector<int32_t> nf(n);
    int64_t in_off = 0, out_off = 0;
    for (int i = 0; i < n; ++i) {
      Part& p = parts[i];
      p.in_off = in_off;
      p.out_off = out_off;
      int64_t t_off = 0;
      for (Ticket* t : p.tickets) {
        for (int ci = 0; ci < srv->cin; ++ci)
          std::memcpy(c.in_host + in_off + (int64_t)ci * p.frames + t_off, &t->in[(size_t)ci * t->frames],
                      t->frames * sizeof(float));
        t_off += t->frames;
      }
      ss[i] = p.st->s;
      din[i] = c.in_dev + in_off;
      dout[i] = c.out_dev + out_off;
      nf[i] = p.frames;
      in_off += (int64_t)srv->cin * p.frames;
      out_off += (int64_t)srv->cout * out_frames_of(srv, p.frames);
    }
    // a large step runs as two concurrent halves launched one by one; other
    // steps replay the context's captured graph (or launch one by one)
    int64_t fa = 0;
    const int h = choose_split(srv->m, n, nf.data(), total, &fa);
    const int cap = (srv->cfg.use_graph && !h) ? srv->cfg.max_streams : n;
    size_t desc_need;
    const int64_t gr = srv->m->plan.input_multiple;
    if (h) {
      const size_t off_b = split_desc_offset(h, fa, gr);
      fill_descriptor(c.desc_host, h, h, ss.data(), din.data(), nf.data(), dout.data(), fa, gr);
      fill_descriptor(c.desc_host + off_b, n - h, n - h, ss.data() + h, din.data() + h, nf.data() + h,
                      dout.data() + h, total - fa, gr);
      desc_need = off_b + desc_bytes(n - h, total - fa, gr);
    } else {
      fill_descriptor(c.desc_host, n, cap, ss.data(), din.data(), nf.data(), dout.data(), total, gr);
      desc_need = desc_bytes(cap, total, gr);
    }
    c.parts = std::move(parts);
    c.out_floats = out_off;
    c.busy = true;
    // enqueue outside the lock: only this thread touches the model and streams
    lk.unlock();
    sc_model* m = srv->m;
    hipError_t e;
    hipStream_t side = nullptr;   // the model's side stream (split steps), read under its lock
    {
      std::lock_guard<std::mutex> g(m->mu);
      e = m->has_last ? hipStreamWaitEvent(srv->hs, m->last_done, 0) : hipSuccess;
      // descriptor and input are read over PCIe by kernels (no DMA hand-off
      // before the step); the output goes back by DMA
      if (e == hipSuccess) e = launch_upload(c.desc_hdev, c.desc_dev, desc_need, srv->hs);
      if (e == hipSuccess) e = launch_upload(c.in_hdev, c.in_dev, in_off * sizeof(float), srv->hs);
      if (e == hipSuccess) e = h ? enqueue_split(m, c.desc_dev, n, h, fa, total, srv->hs) : launch_step(srv, c, n, total);
      if (e == hipSuccess)
        e = hipMemcpyAsync(c.out_host, c.out_dev, out_off * sizeof(float), hipMemcpyDeviceToHost, srv->hs);
      if (e == hipSuccess) e = hipEventRecord(c.done, srv->hs);
      if (e == hipSuccess) {
        m->last_done = c.done;
        m->has_last = true;
        commit_step(n, ss.data(), nf.data());
      }
      side = m->side;
    }
    lk.lock();
    if (e != hipSuccess) {
      srv->worker_error = std::string("step: ") + hipGetErrorString(e);
      for (int i = 0; i < n; ++i) ss[i]->bad = true;
      // finalize the failed context so that waiting callers are released
      // (a split step's second half may still run on the model's side stream)
      hipStreamSynchronize(srv->hs);
      if (side) hipStreamSynchronize(side);
      finalize(srv, c, true);
      continue;
    }
    srv->stats.steps++;
    for (auto& p : c.parts) {
      srv->stats.buffers += (int64_t)p.tickets.size();
      srv->stats.merged_buffers += (int64_t)p.tickets.size() - 1;
      srv->stats.frames_in += p.frames;
      srv->stats.samples_out += srv->cout * out_frames_of(srv, p.frames);
    }
  }
}

// Releases the workspace pin and the model reference taken at creation.
void unpin(sc_server* srv) {
  {
    std::lock_guard<std::mutex> g(srv->m->mu);
    if (srv->cfg.use_graph) srv->m->ws_pins--;
  }
  sc_model_destroy(srv->m);
}

sc_status alloc_ctx(sc_server* srv, StepCtx& c) {
  const int64_t in_f = srv->max_frames * srv->cin;
  const int64_t out_f = out_frames_of(srv, srv->max_frames) * srv->cout;
  const size_t db = desc_bytes(srv->cfg.max_streams, srv->max_frames, srv->m->plan.input_multiple) + kSplitSlack;
  // descriptor and input staging: coherent, read by the upload kernel
  const unsigned flags = hipHostMallocMapped | hipHostMallocCoherent;
  void* dh = nullptr;
  void* ih = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&c.desc_host), db, flags) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c.in_host), in_f * sizeof(float), flags) != hipSuccess ||
      hipHostGetDevicePointer(&dh, c.desc_host, 0) != hipSuccess ||
      hipHostGetDevicePointer(&ih, c.in_host, 0) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&c.out_host), out_f * sizeof(float), hipHostMallocDefault) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c.desc_dev), db) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c.in_dev), in_f * sizeof(float)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&c.out_dev), out_f * sizeof(float)) != hipSuccess ||
      hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess)
    return srv_fail(SC_ENOMEM, "server staging allocation failed");
  c.desc_hdev = static_cast<const unsigned char*>(dh);
  c.in_hdev = static_cast<const float*>(ih);
  return SC_OK;
}

}  // namespace

namespace {

sc_status check_buffer(const sc_server* srv, const float* host_in, int32_t n_frames) {
  if (!host_in) return srv_fail(SC_EINVAL, "null input buffer");
  if (n_frames < 1 || n_frames > srv->cfg.max_buffer_frames || n_frames % srv->m->plan.input_multiple)
    return srv_fail(SC_ELENGTH, "buffer length must be in [1, max_buffer_frames] and a multiple of the total stride");
  return SC_OK;
}

// Whether a buffer for stream_id may be queued now.  Called with srv->mu held.
sc_status check_stream(const sc_server* srv, int64_t stream_id) {
  auto it = srv->streams.find(stream_id);
  if (it != srv->streams.end() && it->second->closing)
    return srv_fail(SC_ESTATE, "stream is closing; wait for its buffers");
  return SC_OK;
}

// Queues one checked buffer.  Called with srv->mu held.
int64_t enqueue_buffer(sc_server* srv, int64_t stream_id, const float* host_in, int32_t n_frames, bool discard,
                       Clock::time_point now) {
  std::unique_ptr<Ticket> t(new Ticket());
  t->stream_id = stream_id;
  t->frames = n_frames;
  t->discard = discard;
  t->in.assign(host_in, host_in + (size_t)srv->cin * n_frames);
  t->t_submit = now;
  auto it = srv->streams.find(stream_id);
  SStream* st;
  if (it == srv->streams.end()) {
    std::unique_ptr<SStream> ns(new SStream());
    ns->id = stream_id;
    st = ns.get();
    srv->streams[stream_id] = std::move(ns);
    srv->waiting.push_back(st);
  } else {
    st = it->second.get();
  }
  t->id = srv->next_ticket++;
  const int64_t id = t->id;
  st->queue.push_back(t.get());
  srv->queued++;
  srv->tickets[id] = std::move(t);
  return id;
}

}  // namespace

extern "C" {

sc_status sc_server_create(sc_model* m, const sc_server_config* cfg, sc_server** out) {
  if (!m || !cfg || !out) return srv_fail(SC_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->max_streams < 1 || cfg->max_buffer_frames < 1 || cfg->max_buffer_frames % m->plan.input_multiple)
    return srv_fail(SC_EINVAL, "max_streams >= 1 and max_buffer_frames a positive multiple of the total stride");
  if (cfg->stream_flags & ~(uint32_t)SC_FLAG_WARMUP_MASK) return srv_fail(SC_EINVAL, "unknown stream flags");
  {
    std::lock_guard<std::mutex> g(m->mu);
    if (m->any_fp8 && !m->have_scales) return srv_fail(SC_EINVAL, "FP8 model has no activation scales");
  }
  std::unique_ptr<sc_server> srv(new sc_server());
  srv->m = m;
  srv->cfg = *cfg;
  srv->cin = m->plan.in_channels;
  srv->cout = m->plan.out_channels;
  srv->out_num = m->plan.out_rate.num;
  srv->out_den = m->plan.out_rate.den;
  srv->max_frames = (int64_t)cfg->max_streams * cfg->max_buffer_frames;
  if (hipSetDevice(m->device) != hipSuccess) return srv_fail(SC_EDEVICE, "hipSetDevice");
  // fixed device memory: workspace for the largest step, staging, descriptors
  {
    std::lock_guard<std::mutex> g(m->mu);
    sc_status st = ensure_workspace(m, srv->max_frames);
    if (st != SC_OK) return st;
    if (cfg->use_graph) m->ws_pins++;   // released by sc_server_destroy
    m->refs++;                          // likewise
  }
  int64_t ws = 0;
  for (const auto& b : m->plan.buf_floats) ws += b.of(m->ws_cap) * 4;
  for (size_t t = 0; t < m->plan.twin_elems.size(); ++t)
    ws += m->plan.twin_elems[t].of(m->ws_cap) * m->plan.twin_esize[t];
  const int64_t staging = kCtx * ((srv->max_frames * srv->cin + out_frames_of(srv.get(), srv->max_frames) * srv->cout) *
                                       4 + (int64_t)(desc_bytes(cfg->max_streams, srv->max_frames,
                                                                m->plan.input_multiple) + kSplitSlack));
  srv->fixed_bytes = ws + staging;
  srv->per_stream_bytes = std::max<int64_t>(m->plan.state_alloc_floats, 1) * 4;
  int64_t fit = cfg->max_streams;
  if (cfg->hbm_budget_bytes > 0) fit = (cfg->hbm_budget_bytes - srv->fixed_bytes) / srv->per_stream_bytes;
  srv->max_admit = (int)std::min<int64_t>(fit, cfg->max_streams);
  if (srv->max_admit < 1) {
    unpin(srv.get());
    return srv_fail(SC_EBUDGET, "HBM budget below the fixed workspace and staging plus one stream");
  }
  if (hipStreamCreateWithFlags(&srv->hs, hipStreamNonBlocking) != hipSuccess) {
    unpin(srv.get());
    return srv_fail(SC_EDEVICE, "hipStreamCreate");
  }
  for (auto& c : srv->ctx) {
    sc_status st = alloc_ctx(srv.get(), c);
    if (st == SC_OK && srv->cfg.use_graph) {
      std::lock_guard<std::mutex> g(srv->m->mu);
      if (capture_step(srv.get(), c) != hipSuccess) st = srv_fail(SC_EDEVICE, "step graph capture failed");
    }
    if (st != SC_OK) {
      for (auto& c2 : srv->ctx) free_ctx(c2);
      hipStreamDestroy(srv->hs);
      unpin(srv.get());
      return st;
    }
  }
  srv->stats.max_admitted = srv->max_admit;
  srv->stats.fixed_bytes = srv->fixed_bytes;
  srv->stats.per_stream_bytes = srv->per_stream_bytes;
  sc_server* raw = srv.release();
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return SC_OK;
}


sc_status sc_server_submit(sc_server* srv, int64_t stream_id, const float* host_in, int32_t n_frames,
                           int64_t* ticket) {
  if (!srv || !ticket) return srv_fail(SC_EINVAL, "null argument");
  sc_status st = check_buffer(srv, host_in, n_frames);
  if (st != SC_OK) return st;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (!srv->worker_error.empty()) return srv_fail(SC_EDEVICE, srv->worker_error);
    st = check_stream(srv, stream_id);
    if (st != SC_OK) return st;
    *ticket = enqueue_buffer(srv, stream_id, host_in, n_frames, false, Clock::now());
  }
  srv->cv.notify_one();
  return SC_OK;
}

sc_status sc_server_submit_batch(sc_server* srv, int32_t n, const int64_t* stream_ids, const float* const* host_in,
                                 const int32_t* n_frames, uint32_t flags, int64_t* tickets) {
  if (!srv || n < 0 || (n > 0 && (!stream_ids || !host_in || !n_frames))) return srv_fail(SC_EINVAL, "null argument");
  if (flags & ~(uint32_t)SC_SUBMIT_DISCARD) return srv_fail(SC_EINVAL, "unknown submit flags");
  const bool discard = flags & SC_SUBMIT_DISCARD;
  if (!tickets && !discard) return srv_fail(SC_EINVAL, "tickets may be NULL only with SC_SUBMIT_DISCARD");
  for (int32_t i = 0; i < n; ++i) {
    sc_status st = check_buffer(srv, host_in[i], n_frames[i]);
    if (st != SC_OK) return st;
  }
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (!srv->worker_error.empty()) return srv_fail(SC_EDEVICE, srv->worker_error);
    for (int32_t i = 0; i < n; ++i) {
      sc_status st = check_stream(srv, stream_ids[i]);
      if (st != SC_OK) return st;
    }
    const auto now = Clock::now();
    for (int32_t i = 0; i < n; ++i) {
      const int64_t id = enqueue_buffer(srv, stream_ids[i], host_in[i], n_frames[i], discard, now);
      if (tickets) tickets[i] = id;
    }
  }
  srv->cv.notify_one();
  return SC_OK;
}

sc_status sc_server_latencies(sc_server* srv, int64_t* tickets, double* latency_s, int64_t max, int64_t* n) {
  if (!srv || !n || max < 0 || (max > 0 && (!tickets || !latency_s))) return srv_fail(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(srv->mu);
  int64_t k = 0;
  while (k < max && !srv->lat_log.empty()) {
    tickets[k] = srv->lat_log.front().first;
    latency_s[k] = srv->lat_log.front().second;
    srv->lat_log.pop_front();
    ++k;
  }
  *n = k;
  return SC_OK;
}

sc_status sc_server_poll(sc_server* srv, int64_t ticket, float* host_out, int64_t out_capacity,
                         double* latency_s) {
  if (!srv) return srv_fail(SC_EINVAL, "null server");
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->tickets.find(ticket);
  if (it == srv->tickets.end()) return srv_fail(SC_EINVAL, "unknown ticket");
  Ticket* t = it->second.get();
  if (!t->done) {
    if (!srv->worker_error.empty()) return srv_fail(SC_EDEVICE, srv->worker_error);
    return SC_PENDING;
  }
  if (t->failed) {
    srv->tickets.erase(it);
    return srv_fail(SC_EDEVICE, srv->worker_error.empty() ? std::string("the buffer's stream saw a failed step")
                                                           : srv->worker_error);
  }
  if (host_out && out_capacity < (int64_t)t->out.size())
    return srv_fail(SC_EINVAL, "host_out holds fewer floats than the buffer's output (" +
                                   std::to_string(t->out.size()) + ")");
  if (host_out) std::memcpy(host_out, t->out.data(), t->out.size() * sizeof(float));
  if (latency_s) *latency_s = std::chrono::duration<double>(t->t_done - t->t_submit).count();
  srv->tickets.erase(it);
  return SC_OK;
}

sc_status sc_server_close_stream(sc_server* srv, int64_t stream_id) {
  if (!srv) return srv_fail(SC_EINVAL, "null server");
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->streams.find(stream_id);
  if (it == srv->streams.end()) return srv_fail(SC_EINVAL, "unknown stream");
  SStream* st = it->second.get();
  st->closing = true;
  if (!st->admitted) {
    // never admitted: its queued buffers still need a slot, keep it waiting
    return SC_OK;
  }
  if (st->queue.empty() && st->inflight == 0) {
    stream_destroy(st->s);
    srv->admitted--;
    srv->streams.erase(it);
  }
  srv->cv.notify_one();
  return SC_OK;
}

sc_status sc_server_drain(sc_server* srv) {
  if (!srv) return srv_fail(SC_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv.notify_one();
  while (srv->queued > 0 && srv->worker_error.empty()) srv->cv_done.wait_for(lk, std::chrono::milliseconds(5));
  if (!srv->worker_error.empty()) return srv_fail(SC_EDEVICE, srv->worker_error);
  return SC_OK;
}

sc_status sc_server_stats_get(sc_server* srv, sc_server_stats* out) {
  if (!srv || !out) return srv_fail(SC_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(srv->mu);
  *out = srv->stats;
  out->admitted = srv->admitted;
  out->waiting = (int32_t)srv->waiting.size();
  out->queued = srv->queued;
  return SC_OK;
}

void sc_server_destroy(sc_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    // buffers of streams that were never admitted cannot complete
    for (SStream* st : srv->waiting) {
      srv->queued -= (int)st->queue.size();
      st->queue.clear();
    }
  }
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  hipSetDevice(srv->m->device);
  hipStreamSynchronize(srv->hs);
  for (auto& kv : srv->streams)
    if (kv.second->s) stream_destroy(kv.second->s);
  {
    // the model must not keep a context's event as its last one (its work is done)
    std::lock_guard<std::mutex> g(srv->m->mu);
    for (auto& c : srv->ctx)
      if (c.done && srv->m->last_done == c.done) {
        srv->m->last_done = nullptr;
        srv->m->has_last = false;
      }
  }
  for (auto& c : srv->ctx) free_ctx(c);
  hipStreamDestroy(srv->hs);
  unpin(srv);
  delete srv;
}

}  // extern "C"
