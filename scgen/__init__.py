"""Seeded synthetic workloads for the streaming convolution path.

This package describes *what is run*: model topologies as plain node lists,
seeded random-init weights, seeded latent inputs and buffer-length draws.  It
holds none of the streaming method's arithmetic (no convolution, no delay
bookkeeping), so both the FP64 oracle and the HIP library can consume it
without sharing any computation.
"""
from .models import (  # noqa: F401
    LRELU_SLOPE,
    stack3,
    decoder,
    rave_decoder_b,
    wide_decoder,
    strided_unit,
    branch_unit,
    encoder,
    autoencoder,
    outconv_unit,
    outconv64_unit,
    outconv48_unit,
    pair48_unit,
    model_by_name,
    n_weights,
    FP8_LAYERS,
    fp8_plan,
)
from .weights import init_weights  # noqa: F401
from .inputs import (  # noqa: F401
    latents, stream_latents, buffer_lengths, split_lengths, random_split, poisson_arrivals, STREAM_SEED_BASE)
