"""Static activation scales for the FP8 path.

The scale of a layer is fixed before streaming starts (a per-buffer scale
would make the output depend on how the input is split): the FP32 path of
the library records max |activated input| of every conv / transposed conv
over a few calibration streams, and the scale is that maximum times a margin.
"""
import numpy as np


def act_scales(sc, model_spec, weights, latents, margin=1.25, device=0):
    """latents: list of float32 arrays [C][T] (one per calibration stream).
    Returns one scale (amax * margin) per conv / transposed-conv node."""
    import torch
    cal = sc.Model(model_spec, weights, "fp32", options=2, device=device)   # FP32 wavefront path
    cal.enable_amax(True)
    for x in latents:
        st = sc.Stream(cal, x.shape[1])
        st.process(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda(device))
        st.close()
    amax = cal.read_amax()
    cal.close()
    return np.maximum(amax * margin, 1e-6).astype(np.float32)
