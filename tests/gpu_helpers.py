"""Helpers for the GPU tests: run the HIP library on seeded inputs and compare
with the FP64 oracle."""
import sys

import numpy as np

import scgen
from oracle import metrics, offline


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def weights_for(name, seed=0):
    m = scgen.model_by_name(name)
    return m, scgen.init_weights(m, seed, "kaiming" if name == "stack3" else "calibrated")


def run_stream(model_obj, x, splits, warmup_mask=False, stream=None):
    """Stream x (numpy [C][T]) through the library in buffers of `splits`;
    returns the concatenated output as numpy float64."""
    import torch
    import paper_2204_07064_amd as sc
    if stream is None:
        stream = sc.Stream(model_obj, max(splits), warmup_mask=warmup_mask)
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    outs = []
    pos = 0
    for n in splits:
        outs.append(stream.process(xd[:, pos:pos + n].contiguous()))
        pos += n
    torch.cuda.synchronize()
    return torch.cat(outs, dim=1).cpu().double().numpy()


def oracle_compare(model, weights, x, s, latency, warmup):
    y = offline.forward(model, weights, x)
    sw, yw = metrics.aligned(s, y, latency, warmup)
    return metrics.max_abs(sw, yw), metrics.snr_db(sw, yw), y
