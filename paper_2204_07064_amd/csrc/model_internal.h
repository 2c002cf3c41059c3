// Internal model / stream objects shared by the runtime and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kernels.h"
#include "sc_internal.h"

namespace sc {

constexpr int kRing = 16;
constexpr size_t kDescHeaderBytes = 64;   // step header: [0] streams, [1] input frames

// Device copies of one op's weights.
struct OpDev {
  void* W = nullptr;        // packed weights (fp32 / bf16 / fp8 by impl)
  float* B = nullptr;       // bias
  float* wscale = nullptr;  // fp8 per-row scales
  int prec = 0;             // precision of this op's kernel
  int32_t win_rows = 0;     // IMPL_WIN: LDS window rows per tile
  int32_t ct_rows = 0, ct_xrows = 0, ct_stash = 0;   // window conv with the transposed conv in its
                                                     // launch: window rows, staged transposed-conv input
                                                     // frames and cache-row pieces per tile
  int32_t pair_rows = 0, pair_arows = 0, pair_stash = 0;   // window conv with the residual conv before it
                                                           // in its launch: its window rows, the first
                                                           // conv's window rows, cache-row pieces per tile
};

// A slot of the descriptor ring: pinned host staging + device copy + event.
// Layout: n Entry records, then one int32 per input frame of the step (its entry).
struct DescSlot {
  unsigned char* host = nullptr;            // coherent pinned memory
  const unsigned char* host_dev = nullptr;  // its device address
  unsigned char* dev = nullptr;
  size_t cap = 0;          // bytes
  hipEvent_t done = nullptr;
  bool pending = false;
};

}  // namespace sc

struct sc_model {
  int device = 0;
  sc_precision prec = SC_FP32;
  uint32_t options = 0;
  sc::Plan plan;
  std::vector<sc::OpDev> opdev;
  std::vector<float> act_scales;   // per layer (FP8)
  bool have_scales = false;
  std::vector<int32_t> layer_prec; // per layer: operand precision 0 FP32, 1 BF16, 2 FP8 e4m3
  bool any_fp8 = false;            // some layer runs on FP8 operands (needs activation scales)
  int32_t n_pairs = 0;             // residual conv pairs run as one launch (fuse_conv_pairs)
  bool input_direct = false;       // the model input's only reader gathers it from the callers'
                                   // buffers: no packing launch (except in calibration runs)
  int64_t weight_bytes = 0;
  // workspace
  std::vector<float*> ws;
  std::vector<void*> tw;           // operand twins
  int64_t ws_cap = 0;              // input frames
  int ws_pins = 0;                 // server graphs holding the workspace's addresses
  // step graph (sc_model_enable_graph): the kernels of one step captured once,
  // sized for graph_streams streams and the whole workspace, reading the
  // descriptor at graph_desc; replayed by every step that fits
  int32_t graph_streams = 0;
  hipGraphExec_t graph_exec = nullptr;
  int64_t graph_frames = 0;        // workspace capacity it was captured for
  unsigned char* graph_desc = nullptr;
  size_t graph_desc_bytes = 0;
  hipStream_t capture_stream = nullptr;
  uint64_t step_gen = 0;           // duplicate-stream check of a step
  // descriptors
  sc::DescSlot ring[sc::kRing];
  int ring_next = 0;
  // cross-stream ordering of steps
  // the event recorded after the model's newest work (every piece of work
  // waits for the previous one, so it covers all of it); not owned: it is a
  // ring slot's, own_done, or a server context's
  hipEvent_t last_done = nullptr;
  bool has_last = false;
  hipEvent_t own_done = nullptr;              // recorded after a state reset
  // a large step runs as two halves of its streams at once: the first on the
  // caller's stream, the second on `side`, joined before the step's event
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // calibration
  float* d_amax = nullptr;
  bool amax_on = false;
  // lifetime: the model itself plus one reference per live stream
  int refs = 1;
  // tracing
  bool prof_on = false;
  std::vector<hipEvent_t> prof_events;        // pool, used in pairs
  size_t prof_used = 0;                       // events recorded since the last fold
  std::vector<int32_t> prof_op;               // op index of each recorded pair
  std::vector<int64_t> prof_in, prof_out, prof_ent;  // per recorded pair
  std::vector<sc_op_profile> prof;            // per op sums
  // offline evaluation (sc_offline_batch, sc_ola_process): the model run on
  // finite buffers with zero padding at both ends, through internal streams
  // whose states sit back to back in one allocation
  std::vector<sc_stream*> off_streams;
  float* off_state = nullptr;                 // off_streams.size() state blocks
  float* off_buf = nullptr;                   // padded inputs and full outputs
  size_t off_cap = 0;                         // floats in off_buf
  hipEvent_t off_done = nullptr;
  std::mutex mu;
};

namespace sc {
// The workspace buffers a launch sequence uses: the model's own (model_ws),
// or regions of the fixed scratch array (stream_process_noalloc).
struct WsView {
  float* const* ws;   // one per plan.buf_floats entry
  void* const* tw;    // one per plan.twin_elems entry
};
inline WsView model_ws(const sc_model* m) { return WsView{m->ws.data(), m->tw.data()}; }
}  // namespace sc

struct sc_stream {
  sc_model* m = nullptr;
  float* d_state = nullptr;
  int32_t max_frames = 0;
  uint32_t flags = 0;
  int64_t pos = 0;
  int parity = 0;
  bool bad = false;
  uint64_t seen = 0;               // step_gen of the last step that listed it
  int64_t end = 0;                 // offline evaluation only (Entry::end); 0 for live streams
};


namespace sc {

// Spare slots after a step's frame -> entry table: kernels read the entry of
// a tile's last frame before they know whether that frame lies in the step
// (a tile spans at most 128 frames, so at most 128 granules at any layer
// rate); the value read there is never used.
constexpr int64_t kFentPad = 256;

// Bytes of a step descriptor for n streams and `frames` input frames; the
// frame -> entry table has one entry per `granule` input frames (the model's
// input multiple: every buffer is a whole number of granules).
inline size_t desc_bytes(int n, int64_t frames, int64_t granule) {  // n: entry capacity
  return kDescHeaderBytes + (size_t)n * sizeof(Entry) +
         (size_t)((frames + granule - 1) / granule + kFentPad) * sizeof(int32_t);
}

// Checks a step's arguments; sets *total to its input frames.  No stream state
// changes (only the duplicate-check marks).
sc_status validate_step(sc_model* m, int n, sc_stream* const* streams, const float* const* d_in,
                        const int32_t* n_frames, float* const* d_out, int64_t* total);
// Writes the step descriptor (header, entries, granule -> entry) into `host`;
// the granule table starts after `ent_capacity` entries (>= n).
void fill_descriptor(unsigned char* host, int n, int ent_capacity, sc_stream* const* streams,
                     const float* const* d_in, const int32_t* n_frames, float* const* d_out, int64_t total,
                     int64_t granule);
// Enqueues the step's kernels on hs reading the descriptor at `dev`; grids are
// sized for grid_n streams and grid_frames input frames (>= the actual step).
// Where a step of n streams splits into two halves that run at once: returns
// the first half's stream count h (0: no split) and sets *f to its frames.
int choose_split(const sc_model* m, int n, const int32_t* n_frames, int64_t total, int64_t* f);
// Byte offset of the second half's descriptor after the first half's.
size_t split_desc_offset(int h, int64_t fa, int64_t granule);
// Launches a split step whose two descriptors are at dev and dev +
// split_desc_offset: the first half on hs, the second on the model's side
// stream, forked from hs and joined back into it.
hipError_t enqueue_split(sc_model* m, const unsigned char* dev, int n, int h, int64_t fa, int64_t total,
                         hipStream_t hs);
// `base`: the input-frame offset at which this launch set's frames sit in the
// workspace (a step's halves use disjoint ranges).
hipError_t enqueue_kernels(sc_model* m, const unsigned char* dev, int grid_n, int64_t grid_frames, hipStream_t hs,
                           int64_t base = 0);
// The same over the workspace buffers `w` instead of the model's own.
hipError_t enqueue_kernels_ws(sc_model* m, const unsigned char* dev, int grid_n, int64_t grid_frames, hipStream_t hs,
                              int64_t base, const WsView& w);
// Once per device, with that device current: resolves the device address of
// the library's fixed scratch array (used by stream_process_noalloc).
hipError_t scratch_setup(int device);
sc_status ensure_workspace(sc_model* m, int64_t frames);
// One batched step (sc_process_batch) with the model's lock held.
sc_status run_step_locked(sc_model* m, int n, sc_stream* const* streams, const float* const* d_in,
                          const int32_t* n_frames, float* const* d_out, hipStream_t hs);
// Records an error message for the calling thread and returns st.
sc_status fail_hip(hipError_t e, const char* what);
// After a successful enqueue: advance positions and flip state copies.
void commit_step(int n, sc_stream* const* streams, const int32_t* n_frames);
sc_status fail_status(sc_status st, const char* msg);

}  // namespace sc
