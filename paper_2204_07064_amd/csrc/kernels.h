// Kernel launch interfaces (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "sc_device.h"

namespace sc {

// Arguments common to the conv-like kernels of one op in one step.
struct LayerArgs {
  const Entry* ents;
  const int32_t* fent;     // entry of every granule (input_multiple input frames) of the step
  const int32_t* hdr;      // device step header: [0] streams, [1] input frames of the step
  int32_t n_ent;           // host: upper bounds used to size grids (the header has the
                           // actual values, so a captured launch serves any smaller step)
  const float* in_buf;     // packed [frames][cin] at the input rate, or null: user input
  const float* in_buf2;    // delay-add second branch
  float* out_buf;          // packed [frames][cout] at the output rate, or null: user output
  const void* W;           // packed weights (layout per kernel)
  const float* B;          // bias [cout]
  const float* wscale;     // FP8: per-output-row weight scale (dequantization)
  float act_scale;         // FP8: static activation scale (amax / 448)
  int32_t cin, cout, k, dil, stride, L, pre_act, post_act, residual, skip_off;
  int32_t A0, A1;
  uint32_t in_num, in_den, out_num, out_den;   // frames per input frame of input / output
  FastDiv fd_in_num, fd_in_den, fd_out_num, fd_out_den, fd_cin, fd_cout;   // fd_*_num: by num * granule
  FastDiv fd_per_ent_narrow;   // L * cin
  int64_t delay;           // output lag (frames at the output rate) for the warm-up mask
  int64_t state_off, state_len, state_off2, state_len2;
  int64_t n_in;            // total input frames of the step at the input rate
  int64_t n_out;           // total output frames of the step at the output rate
  int32_t tile;            // frames per block of the narrow conv kernel (0: per-item kernel)
  // operand twins (see finalize_plan): element type 0 FP32, 1 BF16, 2 FP8 e4m3
  const void* in_twin;     // consumer: pre-activated, pre-rounded input, or null
  void* out_twin;          // producer: twin of the output to write, or null
  float twin_qs;           // producer: scale applied before rounding (FP8: 448 / amax)
  int32_t twin_pre;        // producer: pre-activation of the consumer
  int32_t twin_prec;
  int32_t twin_only;       // producer: the FP32 output has no reader; write the twin only
  int32_t user_in;         // FP32 gathering conv: input rows from each stream's channel-major
                           // buffer (Entry::in, [cin][T]) instead of the packed input
  int64_t tstate_off, tstate_len;   // consumer conv: twin cache copies (floats)
  // window conv only: a one-output-channel stride-1 conv that reads this
  // layer's output and writes the user output, computed in the epilogue
  // (oc.k == 0: none).  Its input frames and rate are this layer's output.
  struct {
    const float* W;        // [k][cin] (cin = this layer's cout)
    const float* B;        // [1]
    int32_t k, dil, L, pre_act, post_act;
    int64_t delay;         // warm-up lag of its output (frames)
    int64_t state_off, state_len;   // its input cache: copies of [L][cin] (floats)
  } oc;
  // window conv only: the transposed conv that produces this layer's input
  // (its output, this layer's input, never reaches memory: each tile computes
  // the frames its window needs from the transposed conv's own input).
  // ct.r == 0: none.
  struct {
    const void* W;         // packed MFMA rows [r * cout][Kpad] (as for its own launch)
    const float* B;        // bias [cout]
    const float* wscale;   // FP8: per-row weight scale
    float act_scale;       // FP8: its static activation scale
    const void* in_twin;   // its input in operand form, [frames][cin] at its input rate
    int32_t r, cin, half_pad, Kpad;
    uint32_t in_num, in_den;   // its input rate (frames per model input frame)
    FastDiv fd_in_den;
    int64_t delay;         // warm-up lag of its output (frames at this layer's input rate)
    int64_t state_off, state_len;   // its carry: copies of [r * cout] (floats)
  } ct;
  // window conv only: the residual window conv whose output is this layer's
  // input, computed in the same launch (its output never reaches memory: each
  // tile computes the frames its window needs from that conv's own input).
  // pa.L == 0: none.  Channels, rates and kernel size equal this layer's.
  struct {
    const void* W;         // packed MFMA rows [cout][Kpad]
    const float* B;        // bias [cout]
    const float* wscale;   // FP8: per-row weight scale
    float act_scale;       // FP8: its static activation scale
    const float* in_buf;   // its input, packed [frames][cin]
    int32_t L, dil, skip_off, pre_act;
    int64_t delay;         // warm-up lag of its output (frames)
    int64_t state_off, state_len;   // its input cache: copies of [L][cin] (floats)
  } pa;
};

// The step descriptor seen through the constant address space: it is
// read-only during a launch, so reads whose address is the same for the
// whole workgroup become scalar loads.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;

// ---- the step's actual size (device header) ----
__device__ inline int32_t step_ents(const LayerArgs& a) { return ((cptr<int32_t>)a.hdr)[0]; }
__device__ inline int32_t step_frames(const LayerArgs& a) { return ((cptr<int32_t>)a.hdr)[1]; }

// ---- rate arithmetic without run-time division ----
// frames of the input / output rate for x input frames of the step
__device__ inline int32_t in_frames(const LayerArgs& a, int32_t x) { return (int32_t)fdiv(a.fd_in_den, (uint32_t)x * a.in_num); }
__device__ inline int32_t out_frames(const LayerArgs& a, int32_t x) { return (int32_t)fdiv(a.fd_out_den, (uint32_t)x * a.out_num); }
// stream (entry) of packed frame n at the input / output rate: the frame
// table has one entry per granule of input frames (fd_*_num divide by the
// rate's numerator times the granule)
__device__ inline int entry_of_in(const LayerArgs& a, int32_t n) { return a.fent[fdiv(a.fd_in_num, (uint32_t)n * a.in_den)]; }
__device__ inline int entry_of_out(const LayerArgs& a, int32_t n) { return a.fent[fdiv(a.fd_out_num, (uint32_t)n * a.out_den)]; }

// Loads and stores through the global address space.  A pointer the
// compiler cannot prove global (read from memory or LDS, or selected between
// two) otherwise becomes a flat access, which also counts on the LDS
// counter: every later wait for an LDS read then waits for it as well, and
// loads meant to be in flight behind LDS work are waited for at once.
// (T: a scalar or a native vector type such as f4 and u4)
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ inline T gload(const void* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline void gstore(void* p, const T& v) {
  *(gptr<T>)p = v;
}

// A stream record read whole: seven 8-byte loads issued together, all
// complete before any field is used (the compiler would otherwise issue each
// field's load in the branch that uses it, one round trip after another).
static_assert(sizeof(Entry) == 56, "Entry is read as seven 8-byte words");
__device__ inline Entry load_entry(const Entry* p) {
  const uint2* src = reinterpret_cast<const uint2*>(p);
  uint2 w[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) w[i] = src[i];
  asm volatile("" ::"v"(w[0]), "v"(w[1]), "v"(w[2]), "v"(w[3]), "v"(w[4]), "v"(w[5]), "v"(w[6]));
  Entry e;
  __builtin_memcpy(&e, w, sizeof(Entry));
  return e;
}

// The streams of a tile of output frames [f0, f0 + F) of a layer: the step's
// output frames, the tile's last frame in the step, its first stream and how
// many streams it touches.  Every wave finds them itself, in one round of
// scalar loads: the step header and the frame-table entries of the tile's
// first frame and of f0 + F - 1 -- read before it is known whether that frame
// lies in the step (the table has spare slots after the step's granules, and
// the value is used only if it does; otherwise the tile ends at the step's
// last stream).  The empty asm keeps the compiler from moving the two table
// reads behind the caller's test of f0 against the step's size.
struct TileSpan {
  int32_t n_cols, f_last, e0, n_seg;
};
__device__ inline TileSpan tile_span(const LayerArgs& a, int32_t f0, int32_t F) {
  const cptr<int32_t> hdr = (cptr<int32_t>)a.hdr;
  const cptr<int32_t> fent = (cptr<int32_t>)a.fent;
  const int32_t n_ent = hdr[0];
  const int32_t n_in = hdr[1];
  const int32_t e0 = fent[fdiv(a.fd_out_num, (uint32_t)f0 * a.out_den)];
  const int32_t e1 = fent[fdiv(a.fd_out_num, (uint32_t)(f0 + F - 1) * a.out_den)];
  asm volatile("" ::"s"(n_ent), "s"(n_in), "s"(e0), "s"(e1));
  TileSpan t;
  t.n_cols = (int32_t)fdiv(a.fd_out_den, (uint32_t)n_in * a.out_num);
  t.f_last = min(f0 + F, t.n_cols) - 1;
  t.e0 = e0;
  t.n_seg = (f0 + F - 1 < t.n_cols ? e1 : n_ent - 1) - e0 + 1;
  return t;
}
// Output frames of stream e that are zeroed, as a range of t * out_den for
// local output frame t: below mask_lo the warm-up mask (absolute output frame
// pos*num/den + t before the layer's delay), from mask_hi on the end of a
// finite signal (offline frame pos*num/den + t - delay at or past end*num/den,
// the layer's output length).  Compared exactly in units of 1/den.
__device__ inline int64_t mask_lo(const Entry& e, int64_t delay, uint32_t num, uint32_t den) {
  return (e.flags & SC_FLAG_WARMUP_MASK) ? delay * (int64_t)den - (int64_t)e.pos * num : INT64_MIN;
}
__device__ inline int64_t mask_hi(const Entry& e, int64_t delay, uint32_t num, uint32_t den) {
  return e.end > 0 ? delay * (int64_t)den + (e.end - e.pos) * (int64_t)num : INT64_MAX;
}
// The same masks as a range of kept local output frames: keep_lo <= t < keep_hi
// (t * den < lo exactly when t < ceil(lo / den); the bounds clamped to int32).
__device__ inline int32_t ceil_frames(int64_t x, uint32_t den) {
  int64_t q = x / (int64_t)den;
  if (x > 0 && q * (int64_t)den != x) ++q;
  return (int32_t)max((int64_t)-1, min(q, (int64_t)INT32_MAX));
}
__device__ inline void keep_range(const Entry& e, int64_t delay, uint32_t num, uint32_t den, int32_t* lo,
                                  int32_t* hi) {
  *lo = ceil_frames(mask_lo(e, delay, num, den), den);
  *hi = ceil_frames(mask_hi(e, delay, num, den), den);
}
__device__ inline bool masked(const LayerArgs& a, const Entry& e, int64_t t) {
  const int64_t x = t * a.out_den;
  return x < mask_lo(e, a.delay, a.out_num, a.out_den) || x >= mask_hi(e, a.delay, a.out_num, a.out_den);
}

__device__ inline int32_t step_in(const LayerArgs& a) { return in_frames(a, step_frames(a)); }
__device__ inline int32_t step_out(const LayerArgs& a) { return out_frames(a, step_frames(a)); }

// Frames per block for the LDS-staged narrow conv (0 if its window does not fit).
int32_t narrow_conv_tile(int cin, int cout, int k, int dil, int stride, int L, int64_t n_out_hint);

hipError_t launch_conv_valu(const LayerArgs& a, hipStream_t s);
// Channel-major user inputs of a step -> packed channels-last [frame][C].
hipError_t launch_pack_input(const Entry* ents, const int32_t* fent, int32_t granule, const int32_t* hdr, int32_t C,
                             int64_t max_frames, float* out, void* twin, int32_t twin_prec, int32_t twin_pre,
                             float twin_qs, hipStream_t s);
hipError_t launch_convt_valu(const LayerArgs& a, hipStream_t s);
hipError_t launch_delay_add(const LayerArgs& a, hipStream_t s);
// max |pre_act(x)| over the step's new input frames of a layer -> atomic max into *amax
hipError_t launch_amax(const LayerArgs& a, float* amax, hipStream_t s);

// MFMA implicit-GEMM kernels for wide layers; prec: 0 FP32, 1 BF16, 2 FP8 e4m3.
hipError_t launch_conv_mfma(const LayerArgs& a, int prec, hipStream_t s);
hipError_t launch_convt_mfma(const LayerArgs& a, int prec, hipStream_t s);
bool conv_mfma_supported(int cin, int cout, int k, int stride, int prec);
// LDS-window MFMA conv: the window rows one tile needs at most (0 if the layer
// does not qualify); min_frames = the fewest frames a stream brings to the layer.
int32_t conv_win_rows(int cin, int cout, int k, int dil, int stride, int L, int64_t min_frames, int prec);
hipError_t launch_conv_win(const LayerArgs& a, int prec, int32_t row_cap, hipStream_t s);
// A window conv with the transposed conv before it computed in the same
// launch (a.ct): whether a layer pair of this shape qualifies (0 if not, else
// the window rows a tile needs; *xrow_cap: the transposed-conv input frames
// a tile stages at most; *stash_cap: the conv's cache-row pieces of 16 bytes
// a tile holds at most), and its launch.
int32_t convt_win_rows(int cin, int cout, int k, int dil, int L, int r, int ct_cin, int prec, int64_t min_frames,
                       int32_t* xrow_cap, int32_t* stash_cap);
hipError_t launch_convt_win(const LayerArgs& a, int prec, int32_t row_cap, int32_t xrow_cap, int32_t stash_cap,
                            hipStream_t s);
// Two residual window convs in one launch (a.pa: the first, whose output only
// the second reads; fuse: the second computes the one-output-channel conv
// after it in its epilogue, a.oc): whether a pair of this shape qualifies (0
// if not, else the second conv's window rows a tile needs; *arow_cap: the
// first conv's window rows, *stash_cap: cache-row pieces of 16 bytes), and
// its launch.
int32_t conv_pair_rows(int c, int k, int dil_a, int dil_b, int prec, int64_t min_frames, bool fuse,
                       int32_t* arow_cap, int32_t* stash_cap);
hipError_t launch_conv_pair(const LayerArgs& a, int prec, int32_t row_cap, int32_t arow_cap, int32_t stash_cap,
                            hipStream_t s);
// Output frames per window tile, and whether a one-output-channel conv of
// k taps, dilation dil (cache L = dil * (k - 1)) can be computed in the
// epilogue of a window conv of this shape.
int32_t conv_win_tile_frames(int cin, int cout);
bool conv_win_out_fusable(int cin, int cout, int k, int dil);
// The frames of such a fused output conv whose taps reach into the previous
// tile of the window conv (its output rows there are in a.in_buf); `a` is the
// output conv's own launch, tile_frames the window conv's tile.
hipError_t launch_conv_out_tail(const LayerArgs& a, int32_t tile_frames, hipStream_t s);
bool convt_mfma_supported(int cin, int cout, int r, int prec);
// The layer that reads the model input on the FP32 MFMA gathering kernel.
bool conv_mfma_fp32_input_supported(int cin, int cout, int k, int stride);
// Host packing of weights into the MFMA kernels' tile order (and, for FP8,
// per-output-row scales).  conv: W[cout][cin][k]; convt: W[cin][cout][2r].
void pack_conv_mfma(const float* w, int cout, int cin, int k, int prec, std::vector<uint8_t>& out,
                    std::vector<float>& wscale);
void pack_convt_mfma(const float* w, int cin, int cout, int r, int prec, std::vector<uint8_t>& out,
                     std::vector<float>& wscale);

// Zero n floats (a kernel rather than a memset so that it is safe to capture
// into a HIP graph).
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
// Copies bytes from src (device-visible pinned host memory or device memory)
// to device memory dst; both 16-byte aligned.
hipError_t launch_upload(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace sc
