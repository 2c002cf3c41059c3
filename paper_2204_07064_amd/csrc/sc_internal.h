// Internal types shared by the planner, the runtime and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "streamconv.h"

namespace sc {

// A non-negative rational number of frames per model-input frame.
struct Frac {
  int64_t num = 1, den = 1;
  static int64_t gcd(int64_t a, int64_t b) {
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a < 0 ? -a : a;
  }
  Frac() = default;
  Frac(int64_t n, int64_t d) : num(n), den(d) { int64_t g = gcd(n, d); if (g) { num /= g; den /= g; } }
  Frac mul(int64_t k) const { return Frac(num * k, den); }
  Frac div(int64_t k) const { return Frac(num, den * k); }
  bool operator==(const Frac& o) const { return num == o.num && den == o.den; }
  // frames of this rate for `t` input frames (t must make it integral)
  int64_t of(int64_t t) const { return t * num / den; }
};

enum OpKind : int32_t { K_CONV = 1, K_CONVT = 2, K_DELAY_ADD = 3 };

// Which kernel family runs an op.
// IMPL_MFMA gathers each K chunk of the operands from HBM; IMPL_WIN stages
// each tile's window rows in LDS once (stride-1 convs with narrow inputs).
// IMPL_TAIL: a one-output-channel conv computed in the epilogue of the window
// conv before it; its own launch only finishes the frames whose taps cross a
// tile boundary of that conv.
enum Impl : int32_t { IMPL_VALU = 0, IMPL_MFMA = 1, IMPL_WIN = 2, IMPL_TAIL = 3 };

// One launch of a processing step (a conv with optional fused residual, a
// transposed conv, or a delay-line sum).
struct Op {
  int32_t kind = 0;
  int32_t impl = IMPL_VALU;
  int32_t node = -1;          // node whose output this op writes
  int32_t conv_node = -1;     // node that owns the weights (conv / convt)
  int32_t src = -1, src2 = -1;
  int32_t cin = 0, cout = 0, k = 0, dil = 1, stride = 1, pad_l = 0, pad_r = 0;
  int32_t pre_act = 0, post_act = 0;
  int32_t residual = 0;       // fused skip: out += raw window row (t + skip_off)
  int32_t skip_off = 0;
  int32_t cache_len = 0;      // conv: cached input frames L; convt: carry frames
  int32_t extra_delay = 0;    // Eq. 2 D_a of a strided conv
  int32_t A0 = 0, A1 = 0;     // delay-line lengths of a delay-add (Eq. 3)
  Frac in_rate, out_rate;
  int64_t out_delay = 0;      // lag of the output stream, in its own frames
  int64_t state_off = 0, state_len = 0;     // floats; copies at off and off + len
  int64_t state_off2 = 0, state_len2 = 0;   // second delay line of a delay-add
  int32_t in_buf = -1, in_buf2 = -1, out_buf = -1;  // workspace buffers; out -1: user output
  int32_t layer = -1;         // index among conv/convt nodes
  int64_t w_off = 0, b_off = 0;             // offsets into the FP32 weight array
  // operand twins: pre-activated, pre-rounded copies of an activation in the
  // MFMA operand type, written by the producer for its single MFMA consumer
  int32_t in_twin = -1;       // consumer: twin buffer of the input
  int32_t out_twin = -1;      // producer: twin buffer it writes
  int32_t twin_pre = 0;       // producer: the consumer's pre-activation
  int32_t twin_layer = -1;    // producer: the consumer's layer (FP8 activation scale)
  int64_t tstate_off = 0, tstate_len = 0;   // consumer conv: twin cache (floats)
  int32_t no_twin = 0;        // an MFMA op that computes in FP32 whatever the model's precision
  int32_t fuse_out = -1;      // window conv: index of the output conv in its epilogue;
                              // IMPL_TAIL op: index of that window conv
  int32_t twin_only = 0;      // producer: its only reader takes the twin and keeps no FP32
                              // input state (a transposed conv), so the FP32 output is not written
  int32_t prec = 0;           // operand precision of this op's kernel: 0 FP32, 1 BF16, 2 FP8 e4m3
  int32_t twin_prec = 0;      // producer: operand precision of the twin's reader
  int32_t convt_in = -1;      // window conv: index of the transposed conv computed in its
                              // launch; that transposed conv: index of the window conv
  int32_t user_in = 0;        // reads the model input from the callers' channel-major buffers
  int32_t pair_in = -1;       // residual window conv: index of the residual window conv before
                              // it, computed in its launch (pair_out: that conv's partner)
  int32_t pair_out = -1;
};

struct Plan {
  std::vector<sc_node> nodes;
  std::vector<Op> ops;
  std::vector<int64_t> delay, warm;
  std::vector<Frac> rate;
  std::vector<int32_t> layer_node;   // conv/convt node of each layer
  std::vector<Frac> buf_floats;      // floats per input frame of each workspace buffer
  int32_t input_buf = -1;            // buffer holding the packed model input
  int32_t input_twin = -1;           // twin of the packed model input
  int32_t input_twin_pre = 0, input_twin_layer = -1;
  std::vector<Frac> twin_elems;      // elements per input frame of each twin buffer
  std::vector<int32_t> twin_esize;   // bytes per element of each twin buffer (its reader's operand type)
  int32_t input_twin_prec = 0;       // operand precision of the input twin's reader
  int32_t in_channels = 0, out_channels = 0;
  int32_t input_multiple = 1;
  Frac out_rate;
  int64_t latency = 0, warmup = 0;
  int64_t state_floats = 0;          // one copy of all state
  int64_t state_alloc_floats = 0;    // both copies, with alignment padding
  int64_t n_weights = 0;
};

// Builds the streaming plan (post-training reconfiguration) of a node list.
sc_status build_plan(const sc_node* nodes, int32_t n, uint32_t options, Plan& plan,
                     std::string& err);

// After the runtime has chosen each op's kernel family and operand precision
// (Op::prec): assigns operand twins (when `twins`) for inputs of MFMA ops that
// have exactly one MFMA reader and a producer that can write them, each in its
// reader's operand type, and lays out the per-stream state (caches, carries,
// delay lines, twin caches).
void finalize_plan(Plan& plan, bool twins);

// Bytes of one operand element of precision 0 (FP32), 1 (BF16) or 2 (FP8).
inline int prec_bytes(int prec) { return prec == 0 ? 4 : (prec == 1 ? 2 : 1); }

void set_error(const std::string& msg);

}  // namespace sc
