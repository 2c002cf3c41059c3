"""Comparison window and error metrics (test infrastructure).

The streamed output s and the offline output y of length T_out agree, after
latency compensation (paper Sec. 4.2), as s[n] = y[n - D] for offline indices
j = n - D in [warmup, T_out - D): the left edge is the warm-up transient of
the zero-initialised caches, the right edge is where the stream has not yet
produced the offline model's last D samples.
"""
import numpy as np


def window(latency, warmup, n_out):
    """Offline index range [lo, hi) compared."""
    return int(warmup), int(n_out) - int(latency)


def aligned(streamed, offline_y, latency, warmup):
    """Return (s_window, y_window) as float64 arrays over the last axis."""
    n_out = offline_y.shape[-1]
    lo, hi = window(latency, warmup, n_out)
    s = np.asarray(streamed, dtype=np.float64)[..., lo + latency:hi + latency]
    y = np.asarray(offline_y, dtype=np.float64)[..., lo:hi]
    return s, y


def max_abs(s, y):
    if s.size == 0:
        return 0.0
    return float(np.max(np.abs(np.asarray(s, np.float64) - np.asarray(y, np.float64))))


def snr_db(s, y):
    """10 log10(sum y^2 / sum (s - y)^2), pooled over every element given."""
    y = np.asarray(y, np.float64)
    e = np.asarray(s, np.float64) - y
    num = float(np.sum(y * y))
    den = float(np.sum(e * e))
    if den == 0.0:
        return float("inf")
    return 10.0 * np.log10(num / den)


def waveform_distance(s, y):
    """Eq. 5: Euclidean distance between raw waveforms."""
    return float(np.linalg.norm(np.asarray(s, np.float64).ravel() - np.asarray(y, np.float64).ravel()))


# STFT of the spectral distance (the paper leaves it unstated): 2048-sample
# frames every 512 samples, periodic Hann analysis window, frames wholly
# inside the signal, amplitude spectrum.
STFT_FFT = 2048
STFT_HOP = 512


def stft_amplitude(x, n_fft=STFT_FFT, hop=STFT_HOP):
    """|STFT| of a 1-D signal: [frames][n_fft // 2 + 1]."""
    x = np.asarray(x, np.float64).ravel()
    if x.size < n_fft:
        return np.zeros((0, n_fft // 2 + 1))
    w = np.sin(np.pi * np.arange(n_fft) / n_fft) ** 2
    starts = np.arange(0, x.size - n_fft + 1, hop)
    frames = np.stack([x[s:s + n_fft] * w for s in starts])
    return np.abs(np.fft.rfft(frames, axis=1))


def spectral_distance(s, y, eps=1.0, n_fft=STFT_FFT, hop=STFT_HOP):
    """Eq. 4: || log(S(s) + eps) - log(S(y) + eps) ||_2 over every STFT
    frame and bin of the amplitude spectra (eps = 1 as the paper sets it)."""
    a = stft_amplitude(s, n_fft, hop)
    b = stft_amplitude(y, n_fft, hop)
    return float(np.linalg.norm(np.log(a + eps) - np.log(b + eps)))
