"""Pins of the overlap-add baseline oracle (paper Sec. 3.3) and of the
spectral distance (Eq. 4) against what the paper and the mathematics fix:
the paper's Hann window, the cross-fade summing to one, special cases whose
overlap-add result is the offline result exactly, the finite receptive field,
and a direct DFT sum."""
import numpy as np
import pytest
from scipy.signal import windows

import scgen
from oracle import metrics, offline, ola


@pytest.mark.parametrize("n", [8, 64, 1000, 4096])
def test_half_overlap_taper_is_the_papers_hann(n):
    # w[n] = sin^2(pi n / N) over the whole buffer = the periodic Hann window
    assert np.allclose(ola.taper(n, n // 2), windows.hann(n, sym=False), atol=1e-15, rtol=0)


def test_zero_overlap_taper_is_rectangular():
    assert np.array_equal(ola.taper(100, 0), np.ones(100))


@pytest.mark.parametrize("window,overlap,spf", [(16, 8, 1), (16, 4, 1), (16, 0, 1), (12, 3, 5), (8, 4, 128)])
def test_tapers_sum_to_one_inside_the_complete_range(window, overlap, spf):
    n_frames = 7 * window + 3
    outs = [np.ones((1, window * spf)) for _ in ola.buffer_starts(n_frames, window, overlap)]
    y = ola.synthesize(outs, window, overlap, spf, n_frames * spf)[0]
    lo, hi = ola.complete_range(n_frames, window, overlap, spf)
    assert hi - lo > window * spf
    assert np.allclose(y[lo:hi], 1.0, atol=1e-12, rtol=0)
    if overlap:
        # the first buffer's rising edge has no partner: faded in from zero
        assert y[0] == 0.0 and np.all(y[:lo] < 1.0)


def _pointwise_model():
    """Every output sample depends on one input frame only: a k=1 conv and a
    transposed conv whose kernel equals its stride (no overlap of its own)."""
    nodes = [{"op": "input", "channels": 2},
             {"op": "conv", "src": 0, "cin": 2, "cout": 3, "k": 1, "dilation": 1, "stride": 1,
              "pad_l": 0, "pad_r": 0, "pre_act": 0, "post_act": 0},
             {"op": "convt", "src": 1, "cin": 3, "cout": 2, "k": 4, "stride": 4, "pad": 0, "pre_act": 1},
             {"op": "conv", "src": 2, "cin": 2, "cout": 1, "k": 1, "dilation": 1, "stride": 1,
              "pad_l": 0, "pad_r": 0, "pre_act": 1, "post_act": 2}]
    return {"name": "pointwise", "nodes": nodes, "in_channels": 2, "out_channels": 1}


@pytest.mark.parametrize("window,overlap", [(16, 8), (16, 4), (16, 0), (10, 5)])
def test_pointwise_model_overlap_add_equals_offline(window, overlap):
    # with no receptive field every buffer reproduces the offline output at
    # its positions, and the cross-fade of equal signals is that signal
    m = _pointwise_model()
    w = scgen.init_weights(m, 3, "kaiming")
    x = scgen.stream_latents(2, 9 * window, 5)
    spf = 4
    y = offline.forward(m, w, x)
    o = ola.overlap_add(m, w, x, window, overlap, spf)
    lo, hi = ola.complete_range(x.shape[1], window, overlap, spf)
    assert np.max(np.abs(o[:, lo:hi] - y[:, lo:hi])) < 1e-12
    # negative control: the buffers placed one frame late do not reproduce it
    outs = ola.buffer_outputs(m, w, x, window, overlap)
    late = ola.synthesize([np.zeros_like(outs[0])] + outs[:-1], window, overlap, spf, x.shape[1] * spf)
    assert np.max(np.abs(late[:, lo + window * spf:hi] - y[:, lo + window * spf:hi])) > 1e-3


def test_single_buffer_without_overlap_is_offline():
    m = scgen.stack3()
    w = scgen.init_weights(m, 0, "kaiming")
    x = scgen.stream_latents(1, 300, 1)
    o = ola.overlap_add(m, w, x, 300, 0, 1)
    assert np.max(np.abs(o - offline.forward(m, w, x))) == 0.0


def test_buffer_interior_is_offline_edges_are_not():
    # the stack's receptive field reaches 1 + 2 + 4 = 7 samples to each side:
    # a buffer's output equals the offline output of the whole signal except
    # within 7 samples of the buffer's edges, where the buffer's own zero
    # padding replaces the neighbouring input (the baseline's artefact)
    m = scgen.stack3()
    w = scgen.init_weights(m, 0, "kaiming")
    x = scgen.stream_latents(1, 640, 2)
    y = offline.forward(m, w, x)
    win = 128
    for k, yk in enumerate(ola.buffer_outputs(m, w, x, win, 0)):
        ref = y[:, k * win:(k + 1) * win]
        assert np.max(np.abs(yk[:, 7:win - 7] - ref[:, 7:win - 7])) < 1e-12
        if k > 0:
            assert np.max(np.abs(yk[:, :7] - ref[:, :7])) > 1e-6
        if k < 640 // win - 1:
            assert np.max(np.abs(yk[:, win - 7:] - ref[:, win - 7:])) > 1e-6


def _dft_amplitude(x, n_fft, hop):
    """|STFT| by the DFT sum written out: X[f][b] = sum_n w[n] x[f hop + n]
    exp(-2 pi i b n / n_fft), periodic Hann w."""
    out = []
    for s in range(0, len(x) - n_fft + 1, hop):
        row = []
        for b in range(n_fft // 2 + 1):
            acc = 0j
            for n in range(n_fft):
                wn = 0.5 - 0.5 * np.cos(2 * np.pi * n / n_fft)
                acc += wn * x[s + n] * np.exp(-2j * np.pi * b * n / n_fft)
            row.append(abs(acc))
        out.append(row)
    return np.array(out)


def test_stft_amplitude_against_the_dft_sum():
    x = np.random.default_rng(0).standard_normal(50)
    a = metrics.stft_amplitude(x, 16, 6)
    assert a.shape == (6, 9)
    assert np.max(np.abs(a - _dft_amplitude(x, 16, 6))) < 1e-12


def test_spectral_distance_special_cases():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(8192)
    assert metrics.spectral_distance(x, x) == 0.0
    # against silence with eps = 1 the distance is || log(1 + S(x)) ||
    ref = np.linalg.norm(np.log1p(metrics.stft_amplitude(x)))
    assert abs(metrics.spectral_distance(x, np.zeros_like(x)) - ref) < 1e-9 * ref
    # a polarity flip leaves the amplitude spectrum alone but not the waveform
    assert metrics.spectral_distance(x, -x) < 1e-9
    assert metrics.waveform_distance(x, -x) == pytest.approx(2.0 * np.linalg.norm(x))
    assert metrics.waveform_distance(x, x + 3.0) == pytest.approx(3.0 * np.sqrt(x.size))
