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
