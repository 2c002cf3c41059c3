"""Offline evaluation on the GPU (the non-causal model on finite buffers,
zero-padded at both ends of every layer, paper Sec. 2.1) and the overlap-add
baseline built on it (Sec. 3.3), against the FP64 oracle; and the paper's
fidelity claim in miniature (Sec. 4.2): the streamed output is the offline
output, the overlap-add output is not."""
import numpy as np
import pytest

import scgen
from oracle import metrics, offline, ola
from gpu_helpers import log, run_stream, weights_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_SNR = 40.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sc():
    import paper_2204_07064_amd as sc
    return sc


@pytest.mark.parametrize("name,lengths", [
    ("stack3", [512, 37, 1]),
    ("rave_b", [16, 5, 1, 33]),
    ("branch3", [40, 7]),
    ("strided", [24, 2]),
    ("strided_aligned", [30]),
    ("outconv", [12, 3]),
    ("encoder", [128 * 12, 128]),
    ("autoencoder", [128 * 16, 128 * 3]),
])
def test_offline_batch_matches_oracle(name, lengths):
    sc = _sc()
    log("offline %s lengths=%s" % (name, lengths))
    m, w = weights_for(name)
    mod = sc.Model(m, w, "fp32")
    xs = [scgen.stream_latents(m["in_channels"], T, 40 + i) for i, T in enumerate(lengths)]
    outs = sc.offline_batch(mod, [torch.from_numpy(x).cuda() for x in xs])
    torch.cuda.synchronize()
    for x, o in zip(xs, outs):
        y = offline.forward(m, w, x)
        g = o.cpu().double().numpy()
        assert g.shape == y.shape
        err = metrics.max_abs(g, y)
        log("  T=%d max-abs %.3e" % (x.shape[1], err))
        assert err <= FP32_TOL


def test_offline_batch_many_buffers_split_step_and_bf16():
    # 40 buffers: the step runs as two concurrent halves of its streams
    sc = _sc()
    m, w = weights_for("rave_b")
    xs = [scgen.stream_latents(16, 16, 100 + i) for i in range(40)]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    ys = [offline.forward(m, w, x) for x in xs]
    o32 = sc.offline_batch(sc.Model(m, w, "fp32"), xd)
    o16 = sc.offline_batch(sc.Model(m, w, "bf16"), xd)
    torch.cuda.synchronize()
    err = max(metrics.max_abs(o.cpu().double().numpy(), y) for o, y in zip(o32, ys))
    snr = metrics.snr_db(np.concatenate([o.cpu().double().numpy() for o in o16], 1), np.concatenate(ys, 1))
    log("offline 40 buffers: fp32 max-abs %.3e, bf16 snr %.1f dB" % (err, snr))
    assert err <= FP32_TOL and snr >= BF16_SNR


@pytest.mark.parametrize("name,frames,window,overlap,spf", [
    ("rave_b", 64, 16, 8, 128),     # 50 %: the paper's Hann window
    ("rave_b", 64, 16, 4, 128),     # 25 %
    ("rave_b", 64, 16, 0, 128),     # 0 %: non-overlapping buffers
    ("rave_b", 61, 8, 4, 128),      # a ragged tail no complete buffer reaches
    ("stack3", 4096, 512, 256, 1),
    ("stack3", 4096, 512, 128, 1),
])
def test_overlap_add_matches_oracle(name, frames, window, overlap, spf):
    sc = _sc()
    log("ola %s frames=%d window=%d overlap=%d" % (name, frames, window, overlap))
    m, w = weights_for(name)
    mod = sc.Model(m, w, "fp32")
    x = scgen.stream_latents(m["in_channels"], frames, 7)
    g = sc.ola_process(mod, torch.from_numpy(x).cuda(), window, overlap)
    torch.cuda.synchronize()
    y = ola.overlap_add(m, w, x, window, overlap, spf)
    err = metrics.max_abs(g.cpu().double().numpy(), y)
    log("  max-abs %.3e" % err)
    assert err <= FP32_TOL


def test_overlap_add_argument_checks():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    x = torch.zeros((16, 32), device="cuda")
    with pytest.raises(sc.ScError):
        sc.ola_process(mod, x, 16, 9)            # overlap above half the window
    # no complete buffer yet: nothing produced
    o = sc.ola_process(mod, x[:, :8].contiguous(), 16, 8)
    torch.cuda.synchronize()
    assert torch.count_nonzero(o).item() == 0


def test_streaming_is_offline_overlap_add_is_not():
    # Sec. 4.2: after latency compensation the streamed output is the offline
    # output (here within FP32 rounding); overlap-add leaves distances that
    # shrink with the overlap but do not vanish
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    frames = 96
    x = scgen.stream_latents(16, frames, 11)
    xd = torch.from_numpy(x).cuda()
    ref = sc.offline_batch(mod, [xd])[0]
    st = sc.Stream(mod, 16, warmup_mask=True)
    s = run_stream(mod, x, scgen.split_lengths(frames, 16), stream=st)
    torch.cuda.synchronize()
    ref = ref.cpu().double().numpy()[0]
    D = mod.latency
    lo, hi = 8 * 128, (frames - 8) * 128        # away from both ends of the signal
    dist = {"stream": metrics.waveform_distance(s[0][lo + D:hi + D], ref[lo:hi])}
    for ov in (8, 4, 0):
        o = sc.ola_process(mod, xd, 16, ov).cpu().double().numpy()[0]
        dist["ola%d" % ov] = metrics.waveform_distance(o[lo:hi], ref[lo:hi])
    log("waveform distances to offline: %s" % dist)
    assert dist["stream"] < 1e-3
    assert min(dist["ola8"], dist["ola4"], dist["ola0"]) > 100 * dist["stream"]
