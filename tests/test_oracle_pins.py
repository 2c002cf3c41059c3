"""Pins of the FP64 oracle against things other than itself (CPU only).

* brute-force pure-Python sums of Eq. 1 (with dilation, stride, padding) and of
  the transposed convolution's scatter definition, on tiny shapes;
* torch.nn.functional conv1d / conv_transpose1d / a whole-graph evaluation in
  float64 on the CPU (a library special case: same definition, other code);
* closed-form latencies and warm-up windows derived by hand (golden file);
* the paper's claims as invariants of the FP64 streaming reference: streamed =
  offline delayed by the latency, for every buffer split (Sec. 4.2);
  alignment delays are needed (negative controls, Sec. 3.1 / 3.2);
* special cases: a delta kernel is a pure delay; k = 1 is a matrix product; a
  linear (activation-free, bias-free) network streams its impulse response.
"""
import itertools
import json
import os

import numpy as np
import pytest
import torch

import scgen
from oracle import metrics, offline, streaming

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# brute force
def brute_conv1d(x, w, b, d, s, pl, pr):
    cin, t = len(x), len(x[0])
    cout, _, k = len(w), len(w[0]), len(w[0][0])

    def xv(ci, i):  # zero padding
        i -= pl
        return x[ci][i] if 0 <= i < t else 0.0
    n_out = (t + pl + pr - d * (k - 1) - 1) // s + 1
    y = []
    for co in range(cout):
        row = []
        for j in range(n_out):
            acc = b[co]
            for ci in range(cin):
                for kk in range(k):
                    acc += w[co][ci][kk] * xv(ci, j * s + d * kk)
            row.append(acc)
        y.append(row)
    return y


def brute_convt(x, w, b, r, p):
    cin, t = len(x), len(x[0])
    _, cout, k = len(w), len(w[0]), len(w[0][0])
    full = [[0.0] * ((t - 1) * r + k) for _ in range(cout)]
    for ci in range(cin):
        for i in range(t):
            for co in range(cout):
                for kk in range(k):
                    full[co][i * r + kk] += w[ci][co][kk] * x[ci][i]
    return [[full[co][j] + b[co] for j in range(p, len(full[co]) - p)] for co in range(cout)]


@pytest.mark.parametrize("cin,cout,t,k,d,s,pl,pr", [
    (1, 1, 9, 3, 1, 1, 1, 1), (3, 2, 17, 3, 2, 1, 2, 2), (2, 4, 20, 5, 3, 1, 6, 6),
    (4, 3, 16, 4, 1, 2, 1, 1), (2, 2, 23, 9, 1, 4, 4, 4), (3, 1, 12, 2, 1, 1, 0, 1),
    (2, 3, 11, 3, 1, 1, 0, 0), (1, 2, 7, 7, 1, 1, 3, 3)])
def test_conv1d_brute_force(cin, cout, t, k, d, s, pl, pr):
    rng = np.random.default_rng(cin * 100 + t)
    x = rng.standard_normal((cin, t))
    w = rng.standard_normal((cout, cin, k))
    b = rng.standard_normal(cout)
    y = offline.conv1d(x, w, b, d, s, pl, pr)
    yb = np.array(brute_conv1d(x.tolist(), w.tolist(), b.tolist(), d, s, pl, pr))
    assert y.shape == yb.shape
    assert np.max(np.abs(y - yb)) <= 1e-12


@pytest.mark.parametrize("cin,cout,t,r", [(1, 1, 5, 2), (3, 2, 7, 4), (2, 3, 4, 8), (4, 2, 1, 2)])
def test_convt_brute_force(cin, cout, t, r):
    rng = np.random.default_rng(cin * 10 + t + r)
    x = rng.standard_normal((cin, t))
    w = rng.standard_normal((cin, cout, 2 * r))
    b = rng.standard_normal(cout)
    y = offline.conv_transpose1d(x, w, b, r, r // 2)
    yb = np.array(brute_convt(x.tolist(), w.tolist(), b.tolist(), r, r // 2))
    assert y.shape == (cout, t * r) == yb.shape
    assert np.max(np.abs(y - yb)) <= 1e-12


# --------------------------------------------------------------------------
# library special case (torch float64 on the CPU)
@pytest.mark.parametrize("cin,cout,t,k,d,s,pl,pr", [
    (16, 32, 64, 3, 9, 1, 9, 9), (8, 8, 40, 4, 1, 2, 1, 1), (5, 7, 33, 7, 1, 1, 3, 3)])
def test_conv1d_vs_torch(cin, cout, t, k, d, s, pl, pr):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((cin, t))
    w = rng.standard_normal((cout, cin, k))
    b = rng.standard_normal(cout)
    y = offline.conv1d(x, w, b, d, s, pl, pr)
    xt = torch.nn.functional.pad(torch.tensor(x)[None], (pl, pr))
    yt = torch.nn.functional.conv1d(xt, torch.tensor(w), torch.tensor(b), stride=s, dilation=d)[0]
    assert y.shape == tuple(yt.shape)
    assert np.max(np.abs(y - yt.numpy())) <= 1e-12


@pytest.mark.parametrize("cin,cout,t,r", [(16, 8, 10, 4), (8, 4, 3, 8), (4, 4, 9, 2)])
def test_convt_vs_torch(cin, cout, t, r):
    rng = np.random.default_rng(8)
    x = rng.standard_normal((cin, t))
    w = rng.standard_normal((cin, cout, 2 * r))
    b = rng.standard_normal(cout)
    y = offline.conv_transpose1d(x, w, b, r, r // 2)
    yt = torch.nn.functional.conv_transpose1d(torch.tensor(x)[None], torch.tensor(w),
                                              torch.tensor(b), stride=r, padding=r // 2)[0]
    assert np.max(np.abs(y - yt.numpy())) <= 1e-12


def torch_forward(model, weights, x):
    """Independent whole-graph evaluation with torch.nn.functional in float64."""
    F = torch.nn.functional
    wt = torch.tensor(np.asarray(weights, np.float64))
    pos = 0
    outs = []
    for nd in model["nodes"]:
        op = nd["op"]
        if op == "input":
            outs.append(torch.tensor(np.asarray(x, np.float64))[None])
            continue
        if op == "add":
            outs.append(outs[nd["src"]] + outs[nd["src2"]])
            continue
        shape = (nd["cout"], nd["cin"], nd["k"]) if op == "conv" else (nd["cin"], nd["cout"], nd["k"])
        n = shape[0] * shape[1] * shape[2]
        w = wt[pos:pos + n].reshape(shape)
        b = wt[pos + n:pos + n + nd["cout"]]
        pos += n + nd["cout"]
        h = outs[nd["src"]]
        if nd["pre_act"] == 1:
            h = F.leaky_relu(h, 0.2)
        if op == "conv":
            h = F.conv1d(F.pad(h, (nd["pad_l"], nd["pad_r"])), w, b, stride=nd["stride"],
                         dilation=nd["dilation"])
            if nd["post_act"] == 2:
                h = torch.tanh(h)
        else:
            h = F.conv_transpose1d(h, w, b, stride=nd["stride"], padding=nd["pad"])
        outs.append(h)
    return outs[-1][0].numpy()


@pytest.mark.parametrize("name,frames", [("stack3", 300), ("rave_b", 12), ("strided", 40),
                                         ("branch", 50), ("branch3", 50), ("encoder", 256), ("outconv", 20),
                                         ("outconv64", 20), ("outconv48", 20)])
def test_forward_vs_torch_graph(name, frames):
    m = scgen.model_by_name(name)
    w = scgen.init_weights(m, 0, "kaiming" if name == "stack3" else "calibrated")
    x = scgen.latents(m["in_channels"], frames, 1)
    y = offline.forward(m, w, x)
    yt = torch_forward(m, w, x)
    assert y.shape == yt.shape
    assert np.max(np.abs(y - yt)) <= 1e-11


# --------------------------------------------------------------------------
# special cases
def test_delta_kernel_is_a_delay():
    # w = e_centre with pads (P, P): y = x; reconfigured causal, stream = x delayed by P
    c, t, k, d = 3, 40, 5, 2
    m = {"name": "delta", "in_channels": c, "out_channels": c, "nodes": [
        {"op": "input", "channels": c},
        {"op": "conv", "src": 0, "cin": c, "cout": c, "k": k, "dilation": d, "stride": 1,
         "pad_l": 4, "pad_r": 4, "pre_act": 0, "post_act": 0}]}
    w = np.zeros((c, c, k), np.float32)
    for i in range(c):
        w[i, i, k // 2] = 1.0
    flat = np.concatenate([w.ravel(), np.zeros(c, np.float32)])
    x = scgen.latents(c, t, 3)
    assert np.array_equal(offline.forward(m, flat, x), x.astype(np.float64))
    s, so = streaming.stream(m, flat, x, [7, 1, 13, 19])
    assert so.latency == 4
    assert np.array_equal(s[:, 4:], x[:, :t - 4].astype(np.float64))
    assert np.all(s[:, :4] == 0)


def test_k1_is_matmul():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6, 30))
    w = rng.standard_normal((4, 6, 1))
    b = rng.standard_normal(4)
    y = offline.conv1d(x, w, b)
    ref = np.einsum("oc,ct->ot", w[:, :, 0], x) + b[:, None]
    assert np.max(np.abs(y - ref)) <= 1e-12


def test_linear_network_impulse_response():
    # no activations, zero biases: the network is LTI; the streamed impulse
    # response equals the offline one shifted by the latency
    m = scgen.rave_decoder_b()
    lin = {"name": "lin", "in_channels": 16, "out_channels": 1,
           "nodes": [dict(nd, pre_act=0, post_act=0) if nd["op"] in ("conv", "convt") else dict(nd)
                     for nd in m["nodes"]]}
    w = scgen.init_weights(lin, 0, "calibrated")
    pos = 0
    for nd in lin["nodes"]:  # zero the biases
        if nd["op"] in ("conv", "convt"):
            pos += nd["cin"] * nd["cout"] * nd["k"]
            w[pos:pos + nd["cout"]] = 0
            pos += nd["cout"]
    frames = 24
    x = np.zeros((16, frames), np.float32)
    x[3, 10] = 1.0
    y = offline.forward(lin, w, x)
    s, so = streaming.stream(lin, w, x, [5, 5, 6, 8])
    D = so.latency
    assert D == 775
    # LTI with exact zeros everywhere before the impulse: no warm-up transient
    assert np.max(np.abs(s[:, D:] - y[:, :y.shape[1] - D])) <= 1e-12
    # shifting the impulse by one frame shifts the output by 128 samples
    x2 = np.zeros_like(x)
    x2[3, 11] = 1.0
    y2 = offline.forward(lin, w, x2)
    assert np.max(np.abs(y2[:, 128 + 900:2800] - y[:, 900:2800 - 128])) <= 1e-12


# --------------------------------------------------------------------------
# closed forms and empirical latency / warm-up
def _golden_delays():
    with open(os.path.join(GOLDEN, "delays.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["stack3", "rave_b", "wide", "strided", "strided_aligned", "branch", "branch3",
                                  "encoder", "autoencoder", "outconv", "outconv64", "outconv48", "pair48"])
def test_latency_and_warmup_closed_form(name):
    g = _golden_delays()[name]
    m = scgen.model_by_name(name)
    so = streaming.StreamingOracle(m, scgen.init_weights(m))
    assert so.latency == g["latency"]
    assert so.warmup == g["warmup"]


@pytest.mark.parametrize("name,frames,buf", [("stack3", 2048, 64), ("rave_b", 48, 5),
                                             ("strided", 64, 6), ("strided_aligned", 64, 4),
                                             ("branch", 60, 7), ("branch3", 61, 5),
                                             ("outconv", 40, 3), ("outconv64", 48, 5), ("outconv48", 40, 3), ("pair48", 40, 3),
                                             ("autoencoder", 128 * 40, 128 * 5)])
def test_latency_and_warmup_empirical(name, frames, buf):
    """Brute-force search: the only lag at which the streamed output matches
    the offline one over the tail is D, and the last mismatching offline index
    is c_L - 1."""
    g = _golden_delays()[name]
    m = scgen.model_by_name(name)
    w = scgen.init_weights(m, 0, "kaiming" if name == "stack3" else "calibrated")
    x = scgen.latents(m["in_channels"], frames, 5)
    y = offline.forward(m, w, x)
    s, so = streaming.stream(m, w, x, scgen.split_lengths(frames, buf))
    n = y.shape[1]
    tail = n // 2
    lags = [lag for lag in range(0, min(n // 4, 4000))
            if np.max(np.abs(s[:, tail:] - y[:, tail - lag:n - lag])) <= 1e-12]
    assert lags == [g["latency"]]
    D = g["latency"]
    err = np.max(np.abs(s[:, D:] - y[:, :n - D]), axis=0)
    # the transient decays to ~1e-10 at its edge: compare at FP64 rounding level
    bad = np.nonzero(err > 1e-13)[0]
    last_bad = int(bad.max()) if bad.size else -1
    assert last_bad + 1 == g["warmup"]


def test_eq2_alignment_property():
    """Eq. 2 makes R + D_c + D_a a multiple of S; the minimal reading is the
    smallest non-negative such delay, the literal one lies in [1, S]."""
    for S, R, Dc in itertools.product(range(1, 6), range(0, 5), range(0, 11)):
        da = streaming.stride_extra_delay(S, R, Dc, "minimal")
        assert (R + Dc + da) % S == 0
        assert 0 <= da < S
        assert all((R + Dc + e) % S != 0 for e in range(da))
        if S > 1:
            dl = streaming.stride_extra_delay(S, R, Dc, "literal")
            assert (R + Dc + dl) % S == 0 and 1 <= dl <= S


def test_eq3_branch_delays():
    assert streaming.branch_delays([1, 4]) == [3, 0]
    assert streaming.branch_delays([5, 5, 2]) == [0, 0, 3]


# --------------------------------------------------------------------------
# invariants of the streaming method (FP64)
def _stream_vs_offline(name, frames, splits, **kw):
    m = scgen.model_by_name(name)
    w = scgen.init_weights(m, 0, "kaiming" if name == "stack3" else "calibrated")
    x = scgen.latents(m["in_channels"], frames, 11)
    y = offline.forward(m, w, x)
    s, so = streaming.stream(m, w, x, splits, **kw)
    sw, yw = metrics.aligned(s, y, so.latency, so.warmup)
    return s, y, so, metrics.max_abs(sw, yw)


@pytest.mark.parametrize("name,frames,mult", [("stack3", 1500, 1), ("rave_b", 40, 1),
                                              ("strided", 60, 2), ("branch", 77, 1),
                                              ("branch3", 83, 1), ("encoder", 512, 128)])
def test_offline_parity_and_split_invariance(name, frames, mult):
    outs = []
    for seed in range(3):
        splits = scgen.random_split(frames, seed, 9, mult)
        s, y, so, err = _stream_vs_offline(name, frames, splits)
        assert err <= 1e-12, (name, splits, err)
        outs.append(s)
    for o in outs[1:]:
        assert np.max(np.abs(o - outs[0])) <= 1e-12


def test_single_frame_buffers_smaller_than_receptive_field():
    # every buffer is one latent frame: far below the 18-frame d=9 cache
    s, y, so, err = _stream_vs_offline("rave_b", 30, [1] * 30)
    assert err <= 1e-12


def test_literal_eq2_reading_also_exact():
    s, y, so, err = _stream_vs_offline("strided", 64, [8] * 8, stride_delay="literal")
    assert err <= 1e-12
    s2, y2, so2, err2 = _stream_vs_offline("strided_aligned", 64, [8] * 8, stride_delay="literal")
    assert err2 <= 1e-12 and so2.latency == 2  # one extra output frame of latency


def test_negative_control_no_stride_alignment():
    s, y, so, err = _stream_vs_offline("strided", 64, [8] * 8, stride_delay="none")
    assert err > 1e-2


@pytest.mark.parametrize("name", ["branch", "branch3", "rave_b"])
def test_negative_control_unaligned_branches(name):
    frames = 24 if name == "rave_b" else 77
    s, y, so, err = _stream_vs_offline(name, frames, [frames], align_branches=False)
    assert err > 1e-2


@pytest.mark.parametrize("name,frames,mult", [("rave_b", 30, 1), ("strided", 40, 2), ("stack3", 700, 1)])
def test_warmup_mask(name, frames, mult):
    splits = scgen.random_split(frames, 4, 7, mult)
    s, y, so, err = _stream_vs_offline(name, frames, splits, warmup_mask=True)
    D = so.latency
    assert so.warmup == 0
    assert np.all(s[:, :D] == 0.0)
    assert np.max(np.abs(s[:, D:] - y[:, :y.shape[1] - D])) <= 1e-12


def test_reset_equals_fresh():
    m = scgen.rave_decoder_b()
    w = scgen.init_weights(m)
    x = scgen.latents(16, 20, 2)
    so = streaming.StreamingOracle(m, w)
    so.process(scgen.latents(16, 7, 9))
    so.reset()
    a = np.concatenate([so.process(x[:, :8]), so.process(x[:, 8:])], axis=1)
    b, _ = streaming.stream(m, w, x, [20])
    assert np.array_equal(a, b) or np.max(np.abs(a - b)) <= 1e-12


# --------------------------------------------------------------------------
# metrics
def test_snr_and_distances():
    y = np.sin(np.linspace(0, 100, 10000))
    e = 1e-3 * np.cos(np.linspace(0, 77, 10000))
    snr = metrics.snr_db(y + e, y)
    assert abs(snr - 10 * np.log10(np.sum(y * y) / np.sum(e * e))) < 1e-9
    assert abs(snr - 60.0) < 0.1      # equal-power sinusoids at 1e-3 amplitude: 60 dB
    assert metrics.max_abs(y + e, y) == pytest.approx(1e-3, rel=1e-6)
    assert metrics.waveform_distance(y + e, y) == pytest.approx(np.sqrt(np.sum(e * e)))
    assert metrics.window(775, 647, 32768) == (647, 31993)
