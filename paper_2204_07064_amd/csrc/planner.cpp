// Host planner: post-training causal reconfiguration of a node list.
//
// For every node it derives (paper Sec. 3):
//   * the cumulative lag D of its stream: a conv adds its right padding R
//     (moved to the left and cached); a conv of stride S first gets the Eq. 2
//     alignment delay D_a = (S - (R + D) mod S) mod S and then lags
//     (D + R + D_a) / S of its own frames (Sec. 3.1); a transposed conv of
//     ratio r and crop p only delays: D -> D*r + p;
//   * branch delays A_i = max_j D_j - D_i for a sum of two branches (Eq. 3);
//   * the warm-up window: the first offline index from which the stream is
//     exact even though later layers start from zero caches;
//   * cache / carry / delay-line lengths and their offsets in the per-stream
//     state block; workspace buffers for intermediate tensors, reused once
//     their last reader has run.
// A sum whose one branch is a stride-1 conv of the other branch becomes a
// single conv op whose skip is the window row P_L (the centre tap): the Eq. 3
// delay of the identity branch is exactly that conv's right padding.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "sc_internal.h"

namespace sc {

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool fail(std::string& err, const char* fmt, int i) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), fmt, i);
  err = buf;
  return false;
}

}  // namespace

sc_status build_plan(const sc_node* nodes, int32_t n, uint32_t options, Plan& plan,
                     std::string& err) {
  plan = Plan();
  if (!nodes || n < 2) { err = "a model needs an input node and at least one layer"; return SC_EINVAL; }
  plan.nodes.assign(nodes, nodes + n);
  const auto& nd = plan.nodes;
  if (nd[0].op != SC_OP_INPUT || nd[0].cout <= 0) { err = "node 0 must be SC_OP_INPUT with cout = channels"; return SC_EINVAL; }

  std::vector<int32_t> chans(n, 0), consumers(n, 0);
  std::vector<bool> clean(n, false);
  plan.delay.assign(n, 0);
  plan.warm.assign(n, 0);
  plan.rate.assign(n, Frac(1, 1));
  std::vector<int32_t> extra(n, 0), cache_len(n, 0), A0(n, 0), A1(n, 0);

  // ---- validation, delays, rates, warm-up --------------------------------
  for (int i = 0; i < n; ++i) {
    const sc_node& x = nd[i];
    if (i == 0) { chans[0] = x.cout; clean[0] = true; continue; }
    if (x.op == SC_OP_INPUT) { fail(err, "node %d: only node 0 may be an input", i); return SC_EINVAL; }
    if (x.src < 0 || x.src >= i) { fail(err, "node %d: src must name an earlier node", i); return SC_EINVAL; }
    consumers[x.src]++;
    const int s = x.src;
    if (x.op == SC_OP_CONV || x.op == SC_OP_CONVT) {
      if (x.cin != chans[s]) { fail(err, "node %d: cin does not match the source's channels", i); return SC_EINVAL; }
      if (x.cout <= 0 || x.k <= 0 || x.stride <= 0) { fail(err, "node %d: cout, k and stride must be positive", i); return SC_EINVAL; }
      if (x.pre_act < 0 || x.pre_act > 1 || x.post_act < 0 || x.post_act > 2 || x.post_act == 1) {
        fail(err, "node %d: pre_act must be NONE/LRELU, post_act NONE/TANH", i); return SC_EINVAL;
      }
      chans[i] = x.cout;
    }
    if (x.op == SC_OP_CONV) {
      if (x.dilation <= 0 || x.pad_l < 0 || x.pad_r < 0) { fail(err, "node %d: bad dilation or padding", i); return SC_EINVAL; }
      const int64_t S = x.stride, R = x.pad_r;
      const int64_t Dc = plan.delay[s];
      const int64_t da = (S - (R + Dc) % S) % S;                 // Eq. 2
      const int64_t L = x.pad_l + R + da;
      if (L < (int64_t)x.dilation * (x.k - 1) - S + 1) {
        fail(err, "node %d: padding too small to stream this conv", i); return SC_EUNSUPPORTED;
      }
      extra[i] = (int32_t)da;
      cache_len[i] = (int32_t)L;
      plan.delay[i] = (Dc + R + da) / S;
      plan.rate[i] = plan.rate[s].div(S);
      plan.warm[i] = clean[s] ? 0 : ceil_div(plan.warm[s] + x.pad_l, S);
      clean[i] = clean[s] && plan.delay[i] == 0;
    } else if (x.op == SC_OP_CONVT) {
      if (x.k != 2 * x.stride || x.pad_l != x.pad_r || x.pad_l < 0 || 2 * x.pad_l > x.k) {
        fail(err, "node %d: transposed conv needs k == 2*stride and a symmetric crop", i); return SC_EUNSUPPORTED;
      }
      const int64_t r = x.stride, p = x.pad_l;
      cache_len[i] = (int32_t)(x.k - r);                           // carried frames
      plan.delay[i] = plan.delay[s] * r + p;
      plan.rate[i] = plan.rate[s].mul(r);
      plan.warm[i] = clean[s] ? 0 : std::max<int64_t>(0, plan.warm[s] * r + x.k - r - p);
      clean[i] = clean[s] && plan.delay[i] == 0;
    } else if (x.op == SC_OP_ADD) {
      if (x.src2 < 0 || x.src2 >= i) { fail(err, "node %d: src2 must name an earlier node", i); return SC_EINVAL; }
      consumers[x.src2]++;
      const int a = x.src, b = x.src2;
      if (chans[a] != chans[b]) { fail(err, "node %d: branches have different channels", i); return SC_EINVAL; }
      if (!(plan.rate[a] == plan.rate[b])) { fail(err, "node %d: branches run at different frame rates", i); return SC_EINVAL; }
      const int64_t top = std::max(plan.delay[a], plan.delay[b]);  // Eq. 3
      A0[i] = (int32_t)(top - plan.delay[a]);
      A1[i] = (int32_t)(top - plan.delay[b]);
      plan.delay[i] = top;
      plan.rate[i] = plan.rate[a];
      plan.warm[i] = std::max(plan.warm[a], plan.warm[b]);
      clean[i] = clean[a] && clean[b];
      chans[i] = chans[a];
    } else {
      fail(err, "node %d: unknown op", i); return SC_EINVAL;
    }
  }
  const int out_node = n - 1;
  plan.in_channels = chans[0];
  plan.out_channels = chans[out_node];
  plan.latency = plan.delay[out_node];
  plan.warmup = plan.warm[out_node];
  plan.out_rate = plan.rate[out_node];
  int64_t mult = 1;
  for (int i = 0; i < n; ++i) {
    const int64_t d = plan.rate[i].den;
    mult = mult / Frac::gcd(mult, d) * d;
  }
  plan.input_multiple = (int32_t)mult;

  // ---- layers and weight offsets ------------------------------------------
  std::vector<int32_t> layer_of(n, -1);
  std::vector<int64_t> w_off(n, 0), b_off(n, 0);
  int64_t pos = 0;
  for (int i = 0; i < n; ++i) {
    if (nd[i].op == SC_OP_CONV || nd[i].op == SC_OP_CONVT) {
      layer_of[i] = (int32_t)plan.layer_node.size();
      plan.layer_node.push_back(i);
      w_off[i] = pos;
      pos += (int64_t)nd[i].cout * nd[i].cin * nd[i].k;
      b_off[i] = pos;
      pos += nd[i].cout;
    }
  }
  plan.n_weights = pos;

  // ---- fusion of residual sums ----------------------------------------------
  std::vector<int32_t> fused_into(n, -1);   // conv node -> add node
  std::vector<int32_t> fused_conv(n, -1);   // add node -> conv node
  if (!(options & SC_MODEL_NO_FUSION)) {
    for (int i = 1; i < n; ++i) {
      if (nd[i].op != SC_OP_ADD) continue;
      for (int side = 0; side < 2; ++side) {
        const int c = side ? nd[i].src2 : nd[i].src;
        const int x = side ? nd[i].src : nd[i].src2;
        const int64_t A_identity = side ? A0[i] : A1[i];
        if (nd[c].op == SC_OP_CONV && nd[c].src == x && nd[c].stride == 1 && nd[c].cin == nd[c].cout &&
            consumers[c] == 1 && c != out_node && fused_into[c] < 0 && A_identity == nd[c].pad_r &&
            nd[c].post_act == SC_ACT_NONE) {
          fused_into[c] = i;
          fused_conv[i] = c;
          break;
        }
      }
    }
  }

  // ---- ops --------------------------------------------------------------------
  std::vector<int32_t> op_of(n, -1);
  for (int i = 1; i < n; ++i) {
    const sc_node& x = nd[i];
    if (fused_into[i] >= 0) continue;
    Op op;
    op.node = i;
    if (x.op == SC_OP_ADD && fused_conv[i] < 0) {
      op.kind = K_DELAY_ADD;
      op.src = x.src;
      op.src2 = x.src2;
      op.cin = op.cout = chans[i];
      op.A0 = A0[i];
      op.A1 = A1[i];
      op.in_rate = plan.rate[x.src];
      op.out_rate = plan.rate[i];
      op.state_len = (int64_t)op.A0 * op.cin;
      op.state_len2 = (int64_t)op.A1 * op.cin;
    } else {
      const int c = (x.op == SC_OP_ADD) ? fused_conv[i] : i;
      const sc_node& cv = nd[c];
      op.kind = (cv.op == SC_OP_CONV) ? K_CONV : K_CONVT;
      op.conv_node = c;
      op.src = cv.src;
      op.cin = cv.cin; op.cout = cv.cout; op.k = cv.k; op.dil = cv.dilation;
      op.stride = cv.stride; op.pad_l = cv.pad_l; op.pad_r = cv.pad_r;
      op.pre_act = cv.pre_act; op.post_act = cv.post_act;
      op.cache_len = cache_len[c];
      op.extra_delay = extra[c];
      op.in_rate = plan.rate[cv.src];
      op.out_rate = plan.rate[c];
      op.layer = layer_of[c];
      op.w_off = w_off[c];
      op.b_off = b_off[c];
      if (op.kind == K_CONV) {
        op.state_len = (int64_t)op.cache_len * op.cin;
        if (x.op == SC_OP_ADD) { op.residual = 1; op.skip_off = cv.pad_l; }
      } else {
        op.state_len = (int64_t)op.cache_len * op.cout;
        op.dil = 1;
      }
    }
    op.out_delay = plan.delay[i];
    op_of[i] = (int32_t)plan.ops.size();
    plan.ops.push_back(op);
  }

  // ---- workspace buffers with reuse after the last reader ---------------------
  std::vector<int32_t> last_use(n, -1);
  for (int o = 0; o < (int)plan.ops.size(); ++o) {
    last_use[plan.ops[o].src] = std::max(last_use[plan.ops[o].src], o);
    if (plan.ops[o].src2 >= 0) last_use[plan.ops[o].src2] = std::max(last_use[plan.ops[o].src2], o);
  }
  std::vector<int32_t> buf_of(n, -1);
  std::vector<bool> busy;
  // the model input is packed channels-last into a workspace buffer first
  if (last_use[0] >= 0) {
    plan.buf_floats.push_back(Frac(chans[0], 1));
    busy.push_back(true);
    buf_of[0] = 0;
    plan.input_buf = 0;
  }
  for (int o = 0; o < (int)plan.ops.size(); ++o) {
    Op& op = plan.ops[o];
    op.in_buf = buf_of[op.src];
    op.in_buf2 = (op.src2 < 0) ? -1 : buf_of[op.src2];
    if (op.node != out_node) {
      const Frac need = plan.rate[op.node].mul(chans[op.node]);
      const double need_d = (double)need.num / need.den;
      int best = -1;
      for (int b = 0; b < (int)plan.buf_floats.size(); ++b) {
        if (busy[b]) continue;
        const double have = (double)plan.buf_floats[b].num / plan.buf_floats[b].den;
        if (have >= need_d && (best < 0 || have < (double)plan.buf_floats[best].num / plan.buf_floats[best].den))
          best = b;
      }
      if (best < 0) {
        best = (int)plan.buf_floats.size();
        plan.buf_floats.push_back(need);
        busy.push_back(false);
      }
      busy[best] = true;
      buf_of[op.node] = best;
      op.out_buf = best;
    }
    // release buffers whose last reader is this op
    for (int i = 0; i < n; ++i)
      if (last_use[i] == o && buf_of[i] >= 0 && i != op.node) busy[buf_of[i]] = false;
  }
  finalize_plan(plan, false);
  return SC_OK;
}

void finalize_plan(Plan& plan, bool twins) {
  const int n = (int)plan.nodes.size();
  // ---- operand twins ----
  plan.twin_elems.clear();
  plan.twin_esize.clear();
  plan.input_twin = -1;
  plan.input_twin_prec = 0;
  for (auto& op : plan.ops) {
    op.in_twin = op.out_twin = -1;
    op.tstate_len = 0;
    op.twin_only = 0;
    op.twin_prec = 0;
  }
  if (twins) {
    std::vector<int> producer(n, -1);
    for (int o = 0; o < (int)plan.ops.size(); ++o) producer[plan.ops[o].node] = o;
    for (int s = 0; s < n; ++s) {
      int reader = -1, n_mfma = 0;
      for (int o = 0; o < (int)plan.ops.size(); ++o) {
        const Op& op = plan.ops[o];
        if (op.impl == IMPL_MFMA && op.src == s) {
          reader = o;
          n_mfma += op.no_twin ? 2 : 1;   // an FP32 reader takes no twin in the model's type
        }
      }
      if (n_mfma != 1) continue;
      const bool from_input = (s == 0 && plan.input_buf >= 0);
      if (!from_input && (producer[s] < 0 || plan.ops[producer[s]].out_buf < 0)) continue;
      const int t = (int)plan.twin_elems.size();
      const int chans = from_input ? plan.in_channels : plan.ops[producer[s]].cout;
      plan.twin_elems.push_back(plan.rate[s].mul(chans));
      Op& rd = plan.ops[reader];
      const int elem_bytes = prec_bytes(rd.prec);
      plan.twin_esize.push_back(elem_bytes);
      rd.in_twin = t;
      if (from_input) {
        plan.input_twin = t;
        plan.input_twin_prec = rd.prec;
        plan.input_twin_pre = rd.pre_act;
        plan.input_twin_layer = rd.layer;
      } else {
        Op& pr = plan.ops[producer[s]];
        pr.out_twin = t;
        pr.twin_prec = rd.prec;
        pr.twin_pre = rd.pre_act;
        pr.twin_layer = rd.layer;
        // a transposed conv reads only the twin (its state is the FP32 carry
        // of its own sums); with no other reader the FP32 output is dead
        int readers = 0;
        for (const Op& o : plan.ops) readers += (o.src == s) + (o.src2 == s);
        if (rd.kind == K_CONVT && readers == 1 && (pr.impl == IMPL_MFMA || pr.impl == IMPL_WIN))
          pr.twin_only = 1;
      }
      if (rd.kind == K_CONV && rd.cache_len > 0)
        rd.tstate_len = ((int64_t)rd.cache_len * rd.cin * elem_bytes + 3) / 4;
    }
  }
  // ---- state layout: double-buffered copies, every region on a 16-float
  // (64-byte) boundary for vector access ----
  auto align16 = [](int64_t x) { return (x + 15) / 16 * 16; };
  int64_t soff = 0, one = 0;
  for (auto& op : plan.ops) {
    op.state_off = soff;
    soff = align16(soff + 2 * op.state_len);
    op.state_off2 = soff;
    soff = align16(soff + 2 * op.state_len2);
    op.tstate_off = soff;
    soff = align16(soff + 2 * op.tstate_len);
    one += op.state_len + op.state_len2;
  }
  plan.state_floats = one;
  plan.state_alloc_floats = soff;
}

}  // namespace sc
