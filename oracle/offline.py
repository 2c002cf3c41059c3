"""Offline FP64 reference model (test infrastructure; see package header).

Every function works on channel-major arrays ``x[c][t]`` in float64 and
follows a plain definition:

* ``conv1d``           -- paper Eq. 1 (Sec. 2.1), the correlation
  y[n][i] = sum_m sum_k w[n][m][k] x[m][i + k], extended with dilation d
  (tap k reads i*S + d*k), stride S (Sec. 2.1) and zero padding of P_L frames
  on the left and P_R on the right (Sec. 2.1).
* ``conv_transpose1d`` -- the transposed convolution of Sec. 2.1: input frame
  i scatters w[i-th input][:, k] into output frame i*r + k, then ``pad``
  frames are cropped on each side (PyTorch ConvTranspose1d semantics).
* ``forward``          -- evaluates a ``scgen`` node list offline.

The per-tap sums use a matrix product as the inner step (sum over input
channels); nothing else is blocked or reordered.
"""
import numpy as np

LRELU_SLOPE = 0.2


def lrelu(x, slope=LRELU_SLOPE):
    """LeakyReLU: x for x >= 0, slope*x otherwise."""
    return np.where(x >= 0, x, slope * x)


def zero_pad(x, pad_l, pad_r):
    """Concatenate pad_l zero frames before and pad_r after x (Sec. 2.1)."""
    c, t = x.shape
    out = np.zeros((c, pad_l + t + pad_r), dtype=np.float64)
    out[:, pad_l:pad_l + t] = x
    return out


def conv1d(x, w, b, dilation=1, stride=1, pad_l=0, pad_r=0):
    """Eq. 1 with dilation, stride and zero padding.

    x: [Cin][T]; w: [Cout][Cin][K]; b: [Cout] (or None).
    y[co][j] = b[co] + sum_ci sum_k w[co][ci][k] * xp[ci][j*S + d*k], with xp
    the zero-padded input, for j in [0, floor((T + P_L + P_R - d(K-1) - 1)/S) + 1).
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cout, cin, k = w.shape
    assert x.shape[0] == cin, (x.shape, w.shape)
    xp = zero_pad(x, pad_l, pad_r)
    n_out = (xp.shape[1] - dilation * (k - 1) - 1) // stride + 1
    if n_out <= 0:
        return np.zeros((cout, 0))
    y = np.zeros((cout, n_out))
    if b is not None:
        y += np.asarray(b, dtype=np.float64)[:, None]
    for kap in range(k):
        first = dilation * kap
        cols = np.ascontiguousarray(xp[:, first:first + stride * (n_out - 1) + 1:stride])
        y += np.ascontiguousarray(w[:, :, kap]) @ cols      # [Cout][Cin] @ [Cin][n_out]
    return y


def transposed_full(x, w, stride):
    """Uncropped, bias-free transposed convolution.

    f[co][i*r + k] = sum over (ci, i, k) of w[ci][co][k] * x[ci][i]; output
    length (T - 1)*r + K.  ``w`` is [Cin][Cout][K] (PyTorch layout).
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    cin, cout, k = w.shape
    assert x.shape[0] == cin
    t = x.shape[1]
    if t == 0:
        return np.zeros((cout, 0))
    f = np.zeros((cout, (t - 1) * stride + k))
    for kap in range(k):
        f[:, kap:kap + stride * (t - 1) + 1:stride] += np.ascontiguousarray(w[:, :, kap].T) @ x
    return f


def conv_transpose1d(x, w, b, stride, pad):
    """Transposed conv with ``pad`` frames cropped on both sides plus bias:
    output length (T - 1)*r + K - 2*pad."""
    f = transposed_full(x, w, stride)
    y = f[:, pad:f.shape[1] - pad].copy()
    if b is not None:
        y += np.asarray(b, dtype=np.float64)[:, None]
    return y


def unpack_weights(model, weights):
    """Split the flat float32 weight array into per-node (W, b) float64 pairs."""
    weights = np.asarray(weights)
    out = {}
    pos = 0
    for i, nd in enumerate(model["nodes"]):
        if nd["op"] == "conv":
            shape = (nd["cout"], nd["cin"], nd["k"])
        elif nd["op"] == "convt":
            shape = (nd["cin"], nd["cout"], nd["k"])
        else:
            continue
        n = shape[0] * shape[1] * shape[2]
        w = weights[pos:pos + n].astype(np.float64).reshape(shape)
        pos += n
        b = weights[pos:pos + nd["cout"]].astype(np.float64)
        pos += nd["cout"]
        out[i] = (w, b)
    assert pos == weights.size, (pos, weights.size)
    return out


def apply_pre(nd, x):
    return lrelu(x) if nd.get("pre_act", 0) == 1 else x


def apply_post(nd, y):
    return np.tanh(y) if nd.get("post_act", 0) == 2 else y


def forward(model, weights, x, return_all=False):
    """Offline forward of a node list on the whole input ``x`` [C][T]."""
    params = unpack_weights(model, weights)
    outs = []
    for i, nd in enumerate(model["nodes"]):
        op = nd["op"]
        if op == "input":
            y = np.asarray(x, dtype=np.float64)
            assert y.shape[0] == nd["channels"]
        elif op == "conv":
            w, b = params[i]
            y = conv1d(apply_pre(nd, outs[nd["src"]]), w, b, nd["dilation"], nd["stride"],
                       nd["pad_l"], nd["pad_r"])
            y = apply_post(nd, y)
        elif op == "convt":
            w, b = params[i]
            y = conv_transpose1d(apply_pre(nd, outs[nd["src"]]), w, b, nd["stride"], nd["pad"])
        elif op == "add":
            a, c = outs[nd["src"]], outs[nd["src2"]]
            assert a.shape == c.shape, (a.shape, c.shape)
            y = a + c
        else:
            raise ValueError(op)
        outs.append(y)
    return outs if return_all else outs[-1]
