"""FP64 CPU oracle for streaming non-causal convolutions -- TEST INFRASTRUCTURE.

This package is the checker, not the product.  Only the test suite, the
smoke entry point and the benchmark's CPU-baseline leg may import it; the HIP
library never calls it and shares no code with it.

* ``offline``   -- the authority: the plain offline model with zero padding
  (the paper's Eq. 1 correlation plus dilation, stride, transposed conv,
  LeakyReLU, tanh, parallel-branch sums), in float64.
* ``streaming`` -- an FP64 buffer-by-buffer implementation of the paper's
  method (Sec. 2.2 cached padding, Sec. 3 post-training causal
  reconfiguration, Sec. 3.1 Eq. 2 stride alignment, Sec. 3.2 Eq. 3 branch
  alignment) used only to self-check the invariants the paper claims
  (streamed output = offline output delayed by the cumulative latency,
  independent of the buffer split, Sec. 4.2).
* ``metrics``   -- comparison window, max-abs, SNR, the spectral distance
  (Eq. 4) and the waveform distance (Eq. 5).
* ``ola``       -- the overlap-add baseline the paper compares with
  (Sec. 3.3): the offline model on each buffer, tapered and summed.

Inputs are float32 arrays (weights and latents from ``scgen``), up-cast to
float64 here.
"""
from . import offline, streaming, metrics, ola  # noqa: F401
