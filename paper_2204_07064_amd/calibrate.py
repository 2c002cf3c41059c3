"""Static activation scales for the FP8 path.

The scale of a layer is fixed before streaming starts (a per-buffer scale
would make the output depend on how the input is split): a calibration model
on the library's FP32 path records max |activated input| of every conv /
transposed conv over a few calibration streams, and the library turns those
maxima into scales (sc_model_calibrated_scales).  This module only drives
that run.
"""
import numpy as np


def act_scales(sc, model_spec, weights, latents, device=0):
    """latents: list of float32 arrays [C][T] (one per calibration stream).
    Returns one static activation scale per conv / transposed-conv node."""
    import torch
    cal = sc.Model(model_spec, weights, "fp32", options=2, device=device)   # FP32 wavefront path
    cal.enable_amax(True)
    for x in latents:
        st = sc.Stream(cal, x.shape[1])
        st.process(torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda(device))
        st.close()
    scales = cal.calibrated_scales()
    cal.close()
    return scales
