"""FP64 buffer-by-buffer reference of the streaming method (test
infrastructure; see package header).

Follows the method in the paper's order:

1. Cached padding (Sec. 2.2, Fig. 1): each convolution keeps the last frames
   of its (activated) input and prepends them to the next buffer instead of
   zero padding.  The cache starts as zeros, which is exactly the left zero
   padding of the offline model.
2. Post-training causal reconfiguration (Sec. 3): the right padding R of a
   layer becomes extra left padding, so the cache holds P_L + R frames and the
   layer's output lags by R frames.
3. Cumulative delay bookkeeping (end of Sec. 3.1): every tensor carries the
   total lag D_c it has accumulated; a stride-1 conv adds R, a transposed conv
   with ratio r and crop p maps D to D*r + p (it only delays, Sec. 3.1).
4. Stride alignment (Sec. 3.1, Eq. 2): before a conv of stride S the input
   gets D_a extra cache frames so that D_c + R + D_a is a multiple of S; the
   output lag is then (D_c + R + D_a)/S.
5. Branch alignment (Sec. 3.2, Eq. 3): branch i of a sum is delayed by
   A_i = max_j D_j - D_i frames through a FIFO of A_i frames.
6. Transposed conv streaming: the uncropped transposed conv of a buffer
   overlaps the next buffer by K - r frames; that tail is carried over and
   added to the next buffer's head (the overlap-add that a transposed conv
   performs internally).

The offline output at index j then appears at stream index j + D (Sec. 4.2:
identical after latency compensation).  ``warmup`` is the first offline index
from which the streamed output is guaranteed exact: before it, the zero
initial caches of later layers stand in for values that the offline model
computes from its own zero padding of *earlier* layers.  With
``warmup_mask=True`` every layer writes exact zeros at stream positions before
its own lag, which removes that transient (warmup = 0).
"""
from fractions import Fraction

import numpy as np

from . import offline


def stride_extra_delay(stride, right_pad, cum_delay, reading="minimal"):
    """Eq. 2: extra input delay D_a that makes R + D_c + D_a a multiple of S.

    The printed formula's operator precedence is ambiguous.  ``"minimal"``
    reads it as (S - ((R + D_c) mod S)) mod S, in [0, S-1]; ``"literal"``
    as S - ((R + D_c) mod S), in [1, S] (one more output frame of latency
    when the lag is already aligned).  Both satisfy the alignment condition.
    """
    s = int(stride)
    if s == 1:
        return 0
    m = (int(right_pad) + int(cum_delay)) % s
    if reading == "minimal":
        return (s - m) % s
    if reading == "literal":
        return s - m
    if reading == "none":          # negative control: no alignment delay
        return 0
    raise ValueError(reading)


def branch_delays(delays):
    """Eq. 3: A_i = max_j D_j - D_i."""
    top = max(delays)
    return [top - d for d in delays]


class StreamingOracle:
    """Streams a ``scgen`` node list buffer by buffer in float64."""

    def __init__(self, model, weights, warmup_mask=False, stride_delay="minimal",
                 align_branches=True):
        self.model = model
        self.nodes = model["nodes"]
        self.params = offline.unpack_weights(model, weights)
        self.mask = bool(warmup_mask)
        self.stride_delay = stride_delay
        self.align_branches = bool(align_branches)
        self._plan()
        self.reset()

    # -- post-training reconfiguration: delays, caches, warm-up -------------
    def _plan(self):
        n = len(self.nodes)
        self.rate = [Fraction(0)] * n      # frames of node i per input frame
        self.delay = [0] * n               # lag D of node i's stream (its frames)
        self.warm = [0] * n                # first exact offline index of node i
        self.clean = [False] * n           # stream positions before D hold exact zeros
        self.extra = [0] * n               # Eq. 2 D_a of a conv
        self.cache_len = [0] * n
        self.align = {}                    # add node -> (A_src, A_src2)
        for i, nd in enumerate(self.nodes):
            op = nd["op"]
            if op == "input":
                self.rate[i] = Fraction(1)
                self.delay[i], self.warm[i], self.clean[i] = 0, 0, True
                continue
            s = nd["src"]
            if op == "conv":
                S, R, PL = nd["stride"], nd["pad_r"], nd["pad_l"]
                d, k = nd["dilation"], nd["k"]
                da = stride_extra_delay(S, R, self.delay[s], self.stride_delay)
                L = PL + R + da
                if L < d * (k - 1) - S + 1:
                    raise ValueError("padding too small to stream node %d" % i)
                self.extra[i] = da
                self.cache_len[i] = L
                self.rate[i] = self.rate[s] / S
                lag = self.delay[s] + R + da
                # without alignment the output lag is fractional; keep the
                # floor so that the negative control can still run
                self.delay[i] = lag // S
                if self.clean[s]:
                    self.warm[i] = 0
                else:
                    self.warm[i] = -(-(self.warm[s] + PL) // S)
                self.clean[i] = self.clean[s] and self.delay[i] == 0
            elif op == "convt":
                r, K, p = nd["stride"], nd["k"], nd["pad"]
                assert K >= r, "transposed conv with K < stride is not streamed"
                self.rate[i] = self.rate[s] * r
                self.delay[i] = self.delay[s] * r + p
                if self.clean[s]:
                    self.warm[i] = 0
                else:
                    self.warm[i] = max(0, self.warm[s] * r + K - r - p)
                self.clean[i] = self.clean[s] and self.delay[i] == 0
            elif op == "add":
                a, b = nd["src"], nd["src2"]
                assert self.rate[a] == self.rate[b], "branches at different rates"
                self.rate[i] = self.rate[a]
                if self.align_branches:
                    A = branch_delays([self.delay[a], self.delay[b]])
                else:
                    A = [0, 0]                  # negative control
                self.align[i] = tuple(A)
                self.delay[i] = max(self.delay[a], self.delay[b])
                self.warm[i] = max(self.warm[a], self.warm[b])
                self.clean[i] = self.clean[a] and self.clean[b]
            else:
                raise ValueError(op)
            if self.mask:
                self.warm[i] = 0
                self.clean[i] = True
        out = n - 1
        self.latency = self.delay[out]
        self.warmup = self.warm[out]
        self.out_rate = self.rate[out]
        # input buffers must produce whole frames at every node
        den = 1
        for r in self.rate:
            den = den * r.denominator // np.gcd(den, r.denominator)
        self.input_multiple = int(den)

    def reset(self):
        self.state = {}
        self.pos = [0] * len(self.nodes)
        for i, nd in enumerate(self.nodes):
            if nd["op"] == "conv":
                self.state[i] = np.zeros((nd["cin"], self.cache_len[i]))
            elif nd["op"] == "convt":
                self.state[i] = np.zeros((nd["cout"], nd["k"] - nd["stride"]))
            elif nd["op"] == "add":
                A = self.align[i]
                srcs = (nd["src"], nd["src2"])
                self.state[i] = [np.zeros((self._channels(srcs[j]), A[j])) for j in range(2)]

    def _channels(self, i):
        nd = self.nodes[i]
        if nd["op"] == "input":
            return nd["channels"]
        if nd["op"] in ("conv", "convt"):
            return nd["cout"]
        return self._channels(nd["src"])

    # -- one buffer ----------------------------------------------------------
    def process(self, x):
        x = np.asarray(x, dtype=np.float64)
        t_in = x.shape[1]
        assert t_in % self.input_multiple == 0, "buffer not a multiple of the total stride"
        outs = []
        for i, nd in enumerate(self.nodes):
            op = nd["op"]
            if op == "input":
                y = x
            elif op == "conv":
                u = offline.apply_pre(nd, outs[nd["src"]])
                v = np.concatenate([self.state[i], u], axis=1)
                w, b = self.params[i]
                n_out = u.shape[1] // nd["stride"]
                assert n_out * nd["stride"] == u.shape[1]
                y = offline.conv1d(v, w, b, nd["dilation"], nd["stride"], 0, 0)[:, :n_out]
                assert y.shape[1] == n_out
                L = self.cache_len[i]
                self.state[i] = v[:, v.shape[1] - L:].copy()
                y = offline.apply_post(nd, y)
            elif op == "convt":
                u = offline.apply_pre(nd, outs[nd["src"]])
                w, b = self.params[i]
                r, K = nd["stride"], nd["k"]
                t = u.shape[1]
                if t == 0:
                    y = np.zeros((nd["cout"], 0))
                else:
                    f = offline.transposed_full(u, w, r)
                    f[:, :K - r] += self.state[i]
                    y = f[:, :t * r] + b[:, None]
                    self.state[i] = f[:, t * r:].copy()
            elif op == "add":
                parts = []
                for j, src in enumerate((nd["src"], nd["src2"])):
                    z = outs[src]
                    A = self.align[i][j]
                    if A > 0:
                        line = np.concatenate([self.state[i][j], z], axis=1)
                        z = line[:, :z.shape[1]]
                        self.state[i][j] = line[:, z.shape[1]:].copy()
                    parts.append(z)
                y = parts[0] + parts[1]
            else:
                raise ValueError(op)
            if self.mask and op != "input":
                start = self.pos[i]
                nz = max(0, min(y.shape[1], self.delay[i] - start))
                if nz:
                    y = y.copy()
                    y[:, :nz] = 0.0
            self.pos[i] += y.shape[1]
            outs.append(y)
        return outs[-1]


def stream(model, weights, x, splits, **kw):
    """Stream ``x`` [C][T] through the model split into buffers of the given
    lengths; returns (concatenated output, oracle)."""
    so = StreamingOracle(model, weights, **kw)
    outs = []
    pos = 0
    for n in splits:
        outs.append(so.process(x[:, pos:pos + n]))
        pos += n
    assert pos == x.shape[1]
    return np.concatenate(outs, axis=1), so
