"""Overlap-add baseline (paper Sec. 3.3), FP64 -- test infrastructure.

The baseline the paper compares its streaming method with: the unmodified
non-causal model is applied to each buffer on its own (zero padding at both
ends of every layer, ``offline.forward``), its output is tapered and added to
the previous buffers' outputs with an offset.

Reading of the paper (it gives the window only for 50 % overlap):

* Buffers hold ``window`` input frames and start every ``hop = window -
  overlap`` frames; the overlap ratio is overlap / window (0.5, 0.25, 0).
* Each buffer's output (window * spf samples, spf = output samples per input
  frame) is multiplied by a taper of the same length that rises over the
  first ``overlap * spf`` samples as sin^2, is 1 in between and falls as the
  mirror image over the last ``overlap * spf`` samples.  At 50 % overlap this
  is the paper's Hann window w[n] = sin^2(pi n / N) over the whole buffer; at
  smaller ratios the same sin^2 edges are compressed into the overlap ("the
  window scaled accordingly"), and at 0 % the taper is all ones
  (non-overlapping buffers, the ablation without cached padding).
* Buffer k's tapered output is added at output sample k * hop * spf.  Where a
  falling edge meets the next buffer's rising edge the two tapers sum to one
  (sin^2 + cos^2), so the output is a cross-fade between neighbouring
  buffers; it is complete from the end of the first rising edge to the start
  of the last falling edge (``complete_range``).

The output is aligned with the offline output sample for sample: the
baseline adds no delay of its own beyond waiting for a whole buffer.
"""
import numpy as np

from . import offline


def taper(win_samples, overlap_samples):
    """The buffer taper: sin^2 rise over the first `overlap_samples`, ones,
    mirrored sin^2 fall over the last `overlap_samples`."""
    n = np.arange(win_samples, dtype=np.float64)
    w = np.ones(win_samples)
    o = int(overlap_samples)
    if o == 0:
        return w
    assert 2 * o <= win_samples, "overlap may not exceed half the buffer"
    rise = n < o
    fall = n >= win_samples - o
    w[rise] = np.sin(np.pi * n[rise] / (2.0 * o)) ** 2
    w[fall] = np.sin(np.pi * (win_samples - n[fall]) / (2.0 * o)) ** 2
    return w


def buffer_starts(n_frames, window, overlap):
    """Input frame at which each complete buffer starts."""
    hop = window - overlap
    assert hop >= 1
    if n_frames < window:
        return []
    return list(range(0, n_frames - window + 1, hop))


def buffer_outputs(model, weights, x, window, overlap):
    """The model applied offline to each buffer on its own: a list of
    [C_out][window * spf] arrays, one per buffer start."""
    return [offline.forward(model, weights, x[:, s:s + window]) for s in buffer_starts(x.shape[1], window, overlap)]


def synthesize(outs, window, overlap, spf, n_out):
    """Taper each buffer output and add it at its start (k * hop * spf):
    the overlap-add output of length n_out samples."""
    hop = window - overlap
    w = taper(window * spf, overlap * spf)
    c = outs[0].shape[0] if outs else 1
    y = np.zeros((c, n_out))
    for k, o in enumerate(outs):
        a = k * hop * spf
        assert o.shape[1] == window * spf, (o.shape, window, spf)
        b = min(a + o.shape[1], n_out)
        y[:, a:b] += o[:, :b - a] * w[:b - a]
    return y


def overlap_add(model, weights, x, window, overlap, spf):
    """The overlap-add baseline over the whole input x [C_in][T]: output
    [C_out][T * spf] (samples after the last complete buffer stay zero)."""
    outs = buffer_outputs(model, weights, x, window, overlap)
    return synthesize(outs, window, overlap, spf, x.shape[1] * spf)


def complete_range(n_frames, window, overlap, spf):
    """Output samples [lo, hi) whose tapers sum to one: after the first
    buffer's rising edge and before the last buffer's falling edge."""
    starts = buffer_starts(n_frames, window, overlap)
    if not starts:
        return 0, 0
    return overlap * spf, (starts[-1] + window - overlap) * spf
