"""Seeded inputs: latents / audio, buffer splits and buffer-length draws.

Values are N(0, 1) float32 (the latent prior of a VAE decoder, and the
white-noise test signal used to time streaming), drawn with NumPy's PCG64.
Stream ``i`` of a multi-stream workload uses seed ``1000 + i``.
"""
import numpy as np

STREAM_SEED_BASE = 1000


def latents(channels, frames, seed):
    """[channels][frames] float32 N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((channels, frames)).astype(np.float32)


def stream_latents(channels, frames, stream_index):
    return latents(channels, frames, STREAM_SEED_BASE + int(stream_index))


def split_lengths(total, buf):
    """Split ``total`` frames into consecutive buffers of ``buf`` (last ragged)."""
    out = []
    left = int(total)
    while left > 0:
        out.append(min(int(buf), left))
        left -= out[-1]
    return out


def buffer_lengths(n, choices, seed, multiple=1):
    """``n`` buffer lengths drawn uniformly from ``choices`` (each a multiple
    of ``multiple``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ch = np.asarray(list(choices), dtype=np.int64)
    assert np.all(ch % multiple == 0)
    return ch[rng.integers(0, len(ch), size=n)].tolist()


def random_split(total, seed, max_buf, multiple=1):
    """A random split of ``total`` frames into buffers of 1..max_buf units of
    ``multiple`` frames (``total`` must be a multiple of ``multiple``)."""
    assert total % multiple == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    left = total // multiple
    while left > 0:
        b = int(rng.integers(1, max_buf + 1))
        b = min(b, left)
        out.append(b * multiple)
        left -= b
    return out


def poisson_arrivals(n, rate, seed):
    """``n`` arrival times (seconds from 0) of a Poisson process of ``rate``
    events per second: cumulative sums of exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))
