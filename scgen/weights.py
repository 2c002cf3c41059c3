"""Seeded random-init weights (float32), no forward passes.

Two modes:

* ``"kaiming"`` -- literal Kaiming-uniform (LeakyReLU 0.2 gain, fan_in =
  cin*k) and zero biases.  Used for the plain 3-layer stack.
* ``"calibrated"`` -- Kaiming-uniform followed by *analytic* per-layer scale
  factors chosen so that a random-init decoder neither saturates its final
  tanh nor decays to zero (either would make precision comparisons
  meaningless).  The factors come from nominal variance bookkeeping on the
  node list (a variance-preserving init keeps the variance of its input;
  an add sums its inputs' variances), never from running the network:

  - a conv whose output is summed back onto its own input (a residual
    branch) is scaled to 0.5 x the RMS of that input;
  - a transposed conv is scaled to unit output RMS;
  - the tanh output conv is scaled to RMS 0.5 before the tanh;
  - biases are U(-0.05, 0.05).

Weights are drawn with NumPy's PCG64 from one seed, layers in node order.
"""
import math

import numpy as np

from .models import LRELU_SLOPE, ACT_LRELU, ACT_TANH

RESIDUAL_BRANCH_RMS = 0.5
PRE_TANH_RMS = 0.5
BIAS_BOUND = 0.05


def _gain(pre_act):
    if pre_act == ACT_LRELU:
        return math.sqrt(2.0 / (1.0 + LRELU_SLOPE ** 2))
    return 1.0


def _residual_branches(nodes):
    """Indices of conv nodes whose output is added back onto their own src."""
    out = set()
    for nd in nodes:
        if nd["op"] != "add":
            continue
        a, b = nd["src"], nd["src2"]
        for c, x in ((a, b), (b, a)):
            if nodes[c]["op"] == "conv" and nodes[c]["src"] == x:
                out.add(c)
    return out


def init_weights(model, seed=0, mode="calibrated"):
    """Return the flat float32 weight array for ``model``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nodes = model["nodes"]
    res = _residual_branches(nodes)
    var = [0.0] * len(nodes)      # nominal variance of each node's output
    chunks = []
    for i, nd in enumerate(nodes):
        op = nd["op"]
        if op == "input":
            var[i] = 1.0
            continue
        if op == "add":
            var[i] = var[nd["src"]] + var[nd["src2"]]
            continue
        cin, cout, k = nd["cin"], nd["cout"], nd["k"]
        if op == "conv":
            fan_in = cin * k
            shape = (cout, cin, k)
        else:  # convt: each output frame sees k/stride taps of every input channel
            fan_in = cin * k // nd["stride"]
            shape = (cin, cout, k)
        gain = _gain(nd["pre_act"]) if mode == "calibrated" else _gain(ACT_LRELU)
        bound = gain * math.sqrt(3.0 / fan_in)
        w = rng.uniform(-bound, bound, size=shape)
        vin = var[nd["src"]]
        scale = 1.0
        if mode == "calibrated":
            if i in res:
                scale = RESIDUAL_BRANCH_RMS
            elif op == "convt":
                scale = 1.0 / math.sqrt(vin)
            elif nd.get("post_act", 0) == ACT_TANH:
                scale = PRE_TANH_RMS / math.sqrt(vin)
            b = rng.uniform(-BIAS_BOUND, BIAS_BOUND, size=(cout,))
        else:
            b = np.zeros((cout,))
        w = w * scale
        # a variance-preserving init keeps vin; the extra factor scales it
        var[i] = vin * scale * scale
        chunks.append(w.astype(np.float32).ravel())
        chunks.append(b.astype(np.float32).ravel())
    if not chunks:
        return np.zeros((0,), np.float32)
    return np.concatenate(chunks).astype(np.float32)
