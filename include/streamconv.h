/*
 * streamconv.h -- C ABI of the MI355X (gfx950) streaming convolution library.
 *
 * The library streams a non-causal 1-D convolutional network buffer by
 * buffer ("Streamable neural audio synthesis with non-causal convolutions",
 * Caillon & Esling, 2022):
 *   - cached padding (Sec. 2.2, Fig. 1): each convolution keeps the last
 *     frames of its input on the device and prepends them to the next buffer;
 *   - post-training causal reconfiguration (Sec. 3): right padding becomes
 *     extra left padding, so every layer lags by its right padding;
 *   - stride alignment (Sec. 3.1, Eq. 2) and parallel-branch alignment
 *     (Sec. 3.2, Eq. 3) with extra delays;
 *   - transposed convolutions streamed with an FP32 overlap carry.
 * The concatenated output of any split of an input into buffers equals the
 * offline (zero-padded) model's output delayed by a fixed latency D
 * (Sec. 4.2), apart from a warm-up transient of the zero-initialised caches
 * (removable with SC_FLAG_WARMUP_MASK).
 *
 * Conventions for every function:
 *   - Device pointers are HIP device memory on the model's device; host
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes and keeps device buffers alive until the HIP stream has passed
 *     the call.  The library owns every object it returns and all device
 *     memory it allocates (weights, per-stream state, workspaces).
 *   - `hip_stream` is a hipStream_t (NULL = the null stream).  Processing
 *     calls are asynchronous on it and return after enqueueing.
 *   - Every function returning sc_status validates its arguments first; on
 *     any error it changes no state and sc_last_error() returns a message
 *     (thread-local, valid until the next failing call on that thread).
 *   - Calls on one sc_stream must be serialized by the caller; different
 *     streams of one model may be driven from different threads (the model
 *     serializes their device work internally).
 */
#ifndef STREAMCONV_H
#define STREAMCONV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sc_model sc_model;    /* immutable after create: plan + device weights */
typedef struct sc_stream sc_stream;  /* one live stream: caches, carries, delay lines */

typedef enum {
  SC_OK = 0,
  SC_EINVAL = -1,       /* bad argument, malformed model */
  SC_ENOMEM = -2,       /* device or host allocation failed */
  SC_EBUDGET = -3,      /* memory budget exhausted */
  SC_ELENGTH = -4,      /* buffer length 0, above the stream's maximum, or not a
                           multiple of the model's total stride */
  SC_EDEVICE = -5,      /* a HIP call or kernel launch failed */
  SC_ESTATE = -6,       /* the stream saw a device error; call stream_reset */
  SC_EUNSUPPORTED = -7, /* valid model that the library cannot stream */
  SC_PENDING = 1        /* sc_server_poll: the buffer is not processed yet */
} sc_status;

typedef enum {
  SC_FP32 = 0,          /* FP32 weights and activations */
  SC_BF16 = 1,          /* BF16 (RNE) conv operands on the wide layers, FP32 accumulate */
  SC_FP8E4M3 = 2        /* OCP FP8 e4m3 conv operands on the wide layers, per-output-
                           channel weight scales, static per-layer activation scales */
} sc_precision;

enum {
  SC_OP_INPUT = 0,
  SC_OP_CONV = 1,       /* Eq. 1 correlation with dilation, stride, zero padding */
  SC_OP_CONVT = 2,      /* transposed conv, kernel 2*stride, crop pad_l == pad_r */
  SC_OP_ADD = 3         /* sum of two parallel branches (Sec. 3.2) */
};

enum { SC_ACT_NONE = 0, SC_ACT_LRELU = 1, SC_ACT_TANH = 2 };  /* LeakyReLU slope 0.2 */

enum {
  SC_FLAG_WARMUP_MASK = 1u  /* every layer writes exact zeros at stream positions
                               before its own latency: the output is then the
                               offline output delayed by D from the first sample,
                               with zeros before D */
};

/* One node of the model graph.  Nodes are listed in evaluation order and
 * node 0 is the input.  Offline semantics (what the stream reproduces):
 *  CONV : y[co][j] = b[co] + sum_ci sum_k W[co][ci][k] * xp[ci][j*stride + dilation*k]
 *         with xp = pre_act(x) zero-padded by pad_l / pad_r (paper Eq. 1 plus
 *         dilation, stride, padding, Sec. 2.1); post_act applied after.
 *         Weights W[cout][cin][k] then b[cout].
 *  CONVT: y = crop_pad(f) + b, f[co][i*stride + k] += W[ci][co][k] * pre_act(x)[ci][i];
 *         k must equal 2*stride and pad_l == pad_r (the crop).  Weights
 *         W[cin][cout][k] (PyTorch layout) then b[cout].
 *  ADD  : y = x[src] + x[src2] (same channels, same frame rate).
 *  INPUT: cout = channels. */
typedef struct {
  int32_t op;
  int32_t src, src2;
  int32_t cin, cout, k, dilation, stride, pad_l, pad_r;
  int32_t pre_act, post_act;
} sc_node;

typedef struct {
  int32_t in_channels, out_channels;
  int32_t out_num, out_den;        /* output frames per input frame (num/den) */
  int32_t input_multiple;          /* input buffer lengths must be multiples of this */
  int32_t n_launch;                /* kernels launched per processing step */
  int64_t latency;                 /* D: output frame n = offline output frame n - D */
  int64_t warmup;                  /* c_L: first offline index guaranteed exact without
                                      SC_FLAG_WARMUP_MASK (0 with it) */
  int64_t state_bytes_per_stream;  /* caches + carries + delay lines, one copy, FP32 */
  int64_t state_alloc_per_stream;  /* bytes actually allocated per stream (double-buffered) */
  int64_t weight_bytes;            /* device bytes of packed weights */
} sc_model_info;

/* Plan a model on the host only (no device work): the post-training
 * reconfiguration of Sec. 3 -- per-node delays, Eq. 2 stride delays, Eq. 3
 * branch delays, cache lengths, latency D and warm-up window.  Fills `out`.
 * Errors: SC_EINVAL (malformed graph), SC_EUNSUPPORTED. */
sc_status sc_plan(const sc_node* nodes, int32_t n_nodes, sc_model_info* out);

/* Build a model on `device`.  `weights` is a host array of n_weights FP32
 * values laid out as described for sc_node.  `act_scales` (host, may be
 * NULL) gives, for SC_FP8E4M3, one static activation scale per CONV/CONVT
 * node in node order (amax of that layer's activated input; NULL = the
 * scales set by sc_model_set_act_scales later, required before processing).
 * Copies everything it needs; the caller may free its arrays on return. */
enum {
  SC_MODEL_NO_FUSION = 1u,  /* run residual sums as explicit delay-line + add kernels
                               instead of the fused centre-tap skip */
  SC_MODEL_NO_MFMA = 2u,    /* run every layer on the FP32 wavefront-FMA kernels
                               (precision must be SC_FP32) */
  SC_MODEL_NO_TWIN = 4u,    /* MFMA layers activate and round their input on load
                               instead of reading the copy their producer wrote in
                               operand form (same results; for testing) */
  SC_MODEL_NO_WIN = 8u,     /* narrow stride-1 MFMA convs gather their operands
                               chunk by chunk instead of staging each tile's
                               [cache | new frames] window in LDS (same results;
                               for testing) */
  SC_MODEL_NO_SPLIT = 16u,  /* run every step as one launch sequence; by default a
                               step of at least 32 streams and 512 input frames runs
                               as two halves of its streams at once, the second on
                               an internal HIP stream joined back into the caller's
                               stream before the step ends (same results; for
                               testing) */
  SC_MODEL_NO_OUT_FUSION = 32u  /* a one-output-channel conv that writes the model
                                   output runs as its own launch; by default it is
                                   computed in the epilogue of an LDS-window conv
                                   that feeds it, and its launch only finishes the
                                   frames whose taps cross that conv's tile
                                   boundaries (same results; for testing) */,
  SC_MODEL_NO_CONVT_FUSION = 64u  /* a transposed conv whose output only the residual
                                   conv after it reads runs as its own launch; by
                                   default that conv's tiles compute the frames
                                   they need in the same launch and the transposed
                                   conv's output never reaches memory (same
                                   results, bitwise; for testing) */,
  SC_MODEL_NO_INPUT_DIRECT = 128u  /* the model input is packed channels-last into
                                   the workspace by its own launch before the first
                                   layer; by default an FP32 MFMA conv that is the
                                   input's only reader gathers it straight from the
                                   callers' channel-major buffers (same results,
                                   bitwise; for testing) */,
  SC_MODEL_NO_PAIR_FUSION = 256u  /* two residual window convs of 64 channels in a
                                   row (the first one's output read only by the
                                   second) run as two launches; by default the
                                   second conv's tiles compute the frames of the
                                   first that their windows need in the same
                                   launch, and the first conv's output never
                                   reaches memory (same results, bitwise; for
                                   testing) */
};
sc_status sc_model_create(const sc_node* nodes, int32_t n_nodes, const float* weights,
                          size_t n_weights, sc_precision precision, const float* act_scales,
                          uint32_t options, int32_t device, sc_model** out);
/* sc_model_create with a precision per layer: `layer_precision` is a host
 * array of sc_model_n_layers values (sc_precision, one per CONV/CONVT node in
 * node order) giving the operand type of that layer's convolution; each
 * producer writes the copy of its output that a reduced-precision reader
 * takes in that reader's type.  Caches, carries, the residual stream and all
 * accumulation stay FP32 in every layer.  A layer that runs on FP32 wavefront
 * FMA in every precision (too few channels, the model input, the model
 * output) stays FP32 whatever its entry.  act_scales as for sc_model_create;
 * they are used by the FP8 layers only.  This is the mixed-precision form of
 * the reduced-precision path: with e4m3's three mantissa bits, one rounding
 * of a full-width layer costs ~28 dB of SNR, so a target above that over
 * many layers in series is met by putting only some layers on FP8.
 * Errors: as sc_model_create; SC_EINVAL also for a null array or an unknown
 * precision in it. */
sc_status sc_model_create_mixed(const sc_node* nodes, int32_t n_nodes, const float* weights,
                                size_t n_weights, const int32_t* layer_precision,
                                const float* act_scales, uint32_t options, int32_t device,
                                sc_model** out);
sc_status sc_model_info_get(const sc_model* model, sc_model_info* out);
/* Number of CONV/CONVT nodes (the length of an act_scales array). */
int32_t sc_model_n_layers(const sc_model* model);
/* Sizes the model's activation workspace for steps of up to `max_step_frames`
 * input frames (summed over the streams of a step).  The workspace otherwise
 * grows on the first step that needs more, which synchronizes the device
 * and reallocates; reserving up front keeps every later step free of that.
 * Errors: SC_EINVAL, SC_ENOMEM, SC_ELENGTH (a server that replays graphs
 * holds the workspace). */
sc_status sc_model_reserve(sc_model* model, int64_t max_step_frames);
/* Steps of up to `max_streams` streams (0: off, the default) replay one
 * hipGraph of the step's kernels instead of launching them one by one.  The
 * graph is captured on first use for the current workspace (grids sized for
 * max_streams streams and the workspace's frames; the kernels read each
 * step's actual size from its descriptor) and captured again after the
 * workspace grows, so reserve the workspace first.  Results are bitwise
 * those of one-by-one launches.  Steps with profiling or calibration enabled
 * launch one by one.  Errors: SC_EINVAL. */
sc_status sc_model_enable_graph(sc_model* model, int32_t max_streams);
/* Replace the static FP8 activation scales (host array, sc_model_n_layers
 * values).  Only between processing calls.  Errors: SC_EINVAL (a scale not
 * positive and finite), SC_ESTATE (a server that replays captured step graphs
 * uses the model: they hold the old scales). */
sc_status sc_model_set_act_scales(sc_model* model, const float* act_scales);
/* Record, for every CONV/CONVT node, max |pre_act(input)| over all frames
 * processed by `model` (an SC_FP32 model) since the last call with reset=1,
 * into the host array `amax_out` (sc_model_n_layers values).  Synchronizes
 * the model's device work. */
sc_status sc_model_read_amax(sc_model* model, float* amax_out, int32_t reset);
/* Turn that recording on or off.  Errors: SC_EINVAL (enable on a model that
 * runs two residual convs in one launch, see SC_MODEL_NO_PAIR_FUSION: the
 * first one's output is never formed; calibrate on an SC_FP32 model). */
sc_status sc_model_enable_amax(sc_model* model, int32_t enable);
/* The static FP8 activation scales calibrated from the maxima recorded so
 * far (as sc_model_read_amax, without reset): for each layer, 1.25 x its
 * max |pre_act(input)| (a margin against peaks the calibration inputs did not
 * reach), at least 1e-6.  Writes sc_model_n_layers values to the host array
 * `scales_out`, ready for sc_model_create's act_scales.  A scale is fixed
 * before streaming starts: a per-buffer scale would make the output depend
 * on how the input is split into buffers.  Synchronizes the model's device
 * work.  Errors: SC_EINVAL, SC_EDEVICE. */
sc_status sc_model_calibrated_scales(sc_model* model, float* scales_out);
/* Releases the caller's reference.  The model's memory is freed once its
 * last stream has been destroyed as well. */
void sc_model_destroy(sc_model* model);

/* Open a stream: allocates and zeroes (on `hip_stream`) its state.  Buffers
 * passed to it may hold 1..max_buffer_frames input frames. */
sc_status stream_create(sc_model* model, int32_t max_buffer_frames, uint32_t flags,
                        void* hip_stream, sc_stream** out);
/* Process one buffer.  d_in: device [in_channels][n_frames] FP32 (channel-
 * major, like a PyTorch NCL tensor without the batch dim).  d_out: device
 * [out_channels][n_frames * out_num / out_den] FP32, fully written.
 * Errors: SC_ELENGTH (no state change), SC_EINVAL, SC_ESTATE, SC_EDEVICE. */
sc_status stream_process(sc_stream* stream, const float* d_in, int32_t n_frames, float* d_out,
                         void* hip_stream);
/* stream_process for callers that cannot allocate device memory while they
 * process (code under HIP graph capture, tight serving loops, hosts that
 * forbid allocation): the same kernels and the same result, bitwise, with the
 * step's workspace (every layer's activations and operand copies) and its
 * descriptor in a fixed device array of SC_NOALLOC_SCRATCH_BYTES that the
 * library holds on each device from load until the process ends, instead of
 * the model's growable workspace.  Calls no hipMalloc / hipFree and no other
 * allocating routine; the stream's own state is the one stream_create made.
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls whose work overlaps on one device (other HIP streams, other
 * models, other threads) race and must be serialized by the caller; ordinary
 * stream_process / sc_process_batch calls do not touch the array.  Never
 * splits the step, never replays a graph, refuses to run while profiling or
 * calibration is on.  Arguments, layouts and ownership as stream_process.
 * Errors: SC_ELENGTH (no state change) also when the buffer's workspace does
 * not fit the array (the message gives the bytes needed; fewer frames per call
 * fit), SC_EINVAL, SC_ESTATE, SC_EDEVICE. */
#define SC_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
sc_status stream_process_noalloc(sc_stream* stream, const float* d_in, int32_t n_frames, float* d_out,
                                 void* hip_stream);
/* Zero all caches, carries and delay lines and the position counter. */
sc_status stream_reset(sc_stream* stream, void* hip_stream);
/* Input frames processed since creation / the last reset. */
int64_t stream_position(const sc_stream* stream);

/* ---- stream state export / import (checkpoint, resume, migration) ----
 * A stream's whole streaming state (every layer's cache, transposed-conv
 * carry and delay line, its position and buffer parity; Sec. 2.2: the cached
 * padding is the only state the method carries between buffers) as a
 * self-describing host byte string.  Importing it into a stream of a model
 * with the same graph and precision (this or another model object, on this
 * or another device) continues the stream bitwise as if the original had
 * processed the following buffers. */
/* Bytes of an exported state for streams of `model`. */
int64_t sc_stream_state_bytes(const sc_model* model);
/* Waits for the stream's queued steps, then writes its state to host memory
 * `host` (`bytes` >= sc_stream_state_bytes).  Errors: SC_EINVAL (null, too
 * small), SC_ESTATE (the stream saw a device error), SC_EDEVICE. */
sc_status stream_export(sc_stream* stream, void* host, int64_t bytes);
/* Replaces the stream's state with an exported one; the stream's own flags
 * and maximum buffer length stay.  Waits for its queued steps first.
 * Errors: SC_EINVAL (null, wrong size, or state of another graph or
 * precision; the stream is left unchanged), SC_EDEVICE. */
sc_status stream_import(sc_stream* stream, const void* host, int64_t bytes);
void stream_destroy(sc_stream* stream);

/* Process one buffer for each of n streams of the same model in one batched
 * pass (one launch per layer for all streams; uneven lengths allowed).  The
 * arrays are host arrays of n entries; each stream may appear at most once.
 * Each stream's result is bitwise identical to processing it alone. */
sc_status sc_process_batch(sc_model* model, int32_t n, sc_stream* const* streams,
                           const float* const* d_in, const int32_t* n_frames,
                           float* const* d_out, void* hip_stream);

/* ---- offline evaluation and the overlap-add baseline ----
 * The model as trained, without streaming: each buffer is a finite signal
 * zero-padded at both ends of every layer (Sec. 2.1), the reference that the
 * streamed output equals after latency compensation (Sec. 4.2).  Runs on the
 * streaming kernels: every layer's output outside the buffer's own span is
 * forced to zero (the padding), and D output samples' worth of zero frames
 * follow the buffer.  Uses internal stream states and a staging buffer owned
 * by the model (grown as needed; growing waits for the device). */
/* n independent buffers: d_in[i] device [in_channels][n_frames[i]] FP32,
 * d_out[i] device [out_channels][n_frames[i] * out_num / out_den] FP32 (fully
 * written, output sample j = the offline output at j; no latency).  n_frames
 * must be whole granules (sc_model_info.input_multiple).  Errors: SC_EINVAL,
 * SC_ELENGTH, SC_ENOMEM, SC_EDEVICE. */
sc_status sc_offline_batch(sc_model* model, int32_t n, const float* const* d_in,
                           const int32_t* n_frames, float* const* d_out, void* hip_stream);
/* The overlap-add baseline of Sec. 3.3 over a whole signal d_in (device
 * [in_channels][n_frames]): buffers of `window` input frames start every
 * window - overlap frames (complete buffers only), each is evaluated offline
 * on its own, multiplied by a taper of window * out_rate samples that rises as
 * sin^2 over the first overlap * out_rate samples, is one in between and
 * falls as the mirror image over the last ones (at overlap = window / 2 the
 * Hann window sin^2(pi n / N) of the paper), and added at its start.  d_out:
 * device [out_channels][n_frames * out_rate], fully written (zero where no
 * complete buffer reaches).  window and overlap are whole granules with
 * 2 * overlap <= window (overlap 0: non-overlapping buffers).  Errors:
 * SC_EINVAL, SC_ELENGTH, SC_ENOMEM, SC_EDEVICE. */
sc_status sc_ola_process(sc_model* model, const float* d_in, int32_t n_frames, int32_t window,
                         int32_t overlap, float* d_out, void* hip_stream);

/* ---- tracing: per-launch timing with HIP events on the processing stream ---- */
typedef struct {
  int32_t kind;        /* 1 conv (with fused skip if residual), 2 transposed conv, 3 delay-line sum */
  int32_t impl;        /* 0 FP32 wavefront FMA, 1 MFMA implicit GEMM (gathered
                          operands), 2 MFMA with LDS-staged windows, 3 the
                          remainder of an output conv computed by the window
                          conv before it (SC_MODEL_NO_OUT_FUSION) */
  int32_t precision;   /* sc_precision of this launch's operands */
  int32_t node;        /* node whose output the launch writes */
  int32_t cin, cout, k, dilation, stride, cache_len, residual;
  int32_t a0, a1;      /* delay-line lengths of a delay-line sum */
  int32_t rate_in_num, rate_in_den, rate_out_num, rate_out_den;  /* frames per input frame */
  double ms;           /* summed event-measured duration since profiling was enabled */
  int64_t launches;    /* launches timed */
  int64_t frames_in;   /* summed input frames (at the launch's input rate) */
  int64_t frames_out;  /* summed output frames (at its output rate) */
  int64_t entries;     /* summed streams over the timed launches */
} sc_op_profile;

/* Enable (1) or disable (0) per-launch timing; enabling clears the sums.
 * While enabled every launch is bracketed by two hipEventRecord calls on the
 * processing stream, and each step first waits on the host for the previous
 * step's timings (the event pool then holds one step's worth). */
sc_status sc_model_profile(sc_model* model, int32_t enable);
/* Synchronizes, then fills up to `max_ops` records (one per launch of a
 * step, in launch order) and sets *n_ops to the number of launches per step. */
sc_status sc_model_profile_read(sc_model* model, sc_op_profile* out, int32_t max_ops, int32_t* n_ops);

/* ---- serving: continuous batching of many live streams ----
 * A server holds a reference to its model and owns one worker thread and one
 * HIP stream.  Other processing calls on the same model stay legal and are
 * ordered with the server's steps; while a server that replays graphs lives,
 * a call whose step needs a larger workspace than the server's (max_streams *
 * max_buffer_frames input frames) fails with SC_ELENGTH.  Buffers submitted for any number of streams
 * are queued; every step the worker takes the next buffer of each admitted
 * stream (merging further queued buffers of the same stream up to
 * max_buffer_frames, which the split invariance of the method makes exact),
 * runs them as one batched step, and stamps each buffer's latency from
 * submission to completion.  Buffers arriving while a step runs join the
 * next one.  Streams are admitted first come first served while a slot and
 * the HBM budget (per-stream state, fixed workspace and staging) allow; the
 * others wait until a stream is closed.  Results are bitwise those of
 * processing each stream alone. */
typedef struct sc_server sc_server;
typedef struct {
  int32_t max_streams;        /* slots: streams admitted at once */
  int32_t max_buffer_frames;  /* per stream per step (also the largest buffer accepted) */
  int64_t hbm_budget_bytes;   /* device memory the server may use (0: no limit) */
  int32_t use_graph;          /* 1: replay one hipGraph per step context, captured by
                                 sc_server_create on the calling thread; steps large
                                 enough to split (SC_MODEL_NO_SPLIT) launch one by one */
  uint32_t stream_flags;      /* SC_FLAG_* applied to every stream */
} sc_server_config;
typedef struct {
  int64_t steps, buffers, merged_buffers, frames_in, samples_out;
  int32_t admitted, waiting, max_admitted, queued;
  int64_t fixed_bytes, per_stream_bytes;
} sc_server_stats;

/* Errors: SC_EINVAL, SC_EBUDGET (budget below the fixed memory and one
 * stream), SC_ENOMEM, SC_EDEVICE (stream creation or graph capture failed). */
sc_status sc_server_create(sc_model* model, const sc_server_config* config, sc_server** out);
/* Queue one buffer (host memory [in_channels][n_frames], copied) of stream
 * `stream_id`; the stream is opened on first use.  Sets *ticket. */
sc_status sc_server_submit(sc_server* server, int64_t stream_id, const float* host_in, int32_t n_frames,
                           int64_t* ticket);
/* Flags of sc_server_submit_batch. */
enum {
  SC_SUBMIT_DISCARD = 1u  /* keep no output: at completion the ticket is forgotten
                             and (ticket, latency) goes to the latency log */
};
/* Queues n buffers in order (buffer i: stream stream_ids[i], host memory
 * host_in[i] of [in_channels][n_frames[i]], copied) under one lock, which
 * keeps the per-buffer cost low for load generators.  All buffers are checked
 * first: on an error none is queued.  Sets tickets[i] (may be NULL with
 * SC_SUBMIT_DISCARD). */
sc_status sc_server_submit_batch(sc_server* server, int32_t n, const int64_t* stream_ids,
                                 const float* const* host_in, const int32_t* n_frames, uint32_t flags,
                                 int64_t* tickets);
/* Moves up to `max` entries of the latency log (buffers submitted with
 * SC_SUBMIT_DISCARD, in completion order) to tickets[] / latency_s[]
 * (seconds from submission to completion) and sets *n to their number. */
sc_status sc_server_latencies(sc_server* server, int64_t* tickets, double* latency_s, int64_t max, int64_t* n);
/* SC_OK: done -- copies the output ([out_channels][n_frames * out_num / out_den])
 * to host_out (may be NULL; it holds out_capacity floats) and the
 * submit-to-completion latency in seconds to *latency_s (may be NULL), and
 * forgets the ticket.  SC_PENDING: not yet.  SC_EINVAL: unknown ticket, or
 * host_out holds fewer floats than the output (the ticket is kept).
 * SC_EDEVICE: the buffer's step failed, or its stream saw a failed step
 * before it (the ticket is forgotten). */
sc_status sc_server_poll(sc_server* server, int64_t ticket, float* host_out, int64_t out_capacity,
                         double* latency_s);
/* No more buffers for this stream: its slot is freed once its queued buffers
 * are done (a later submit with the same id opens a new stream). */
sc_status sc_server_close_stream(sc_server* server, int64_t stream_id);
/* Blocks until every queued buffer is processed. */
sc_status sc_server_drain(sc_server* server);
sc_status sc_server_stats_get(sc_server* server, sc_server_stats* out);
void sc_server_destroy(sc_server* server);

const char* sc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STREAMCONV_H */
