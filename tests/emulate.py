"""CPU emulation of the reduced-precision operand rounding (test helper).

The library rounds the operands of its MFMA layers: BF16 (round to nearest
even) weights and activated inputs, or OCP FP8 e4m3 with a per-output-row
weight scale max|W_row|/448 and a static activation scale amax/448.  This
module evaluates the offline model in float64 on the same rounded operands
(rounding through torch's bfloat16 / float8_e4m3fn casts), so the GPU result
can be checked against the intended arithmetic much more tightly than
against the unrounded FP64 oracle.
"""
import numpy as np
import torch

from oracle import offline


def mfma_layer(nd, is_last, reads_input=False, precision="bf16"):
    """Mirror of the library's rule for which layers run on MFMA (every layer
    reads a packed workspace buffer; the last one writes the user's output)."""
    if is_last:
        return False
    es = {"fp32": 4, "bf16": 2, "fp8": 1}[precision]
    if nd["op"] == "conv":
        return (nd["stride"] == 1 and nd["cin"] * es % 16 == 0 and nd["cin"] % 8 == 0 and nd["cout"] % 16 == 0
                and nd["cin"] >= 32 and nd["cout"] >= 32)
    if nd["op"] == "convt":
        m = nd["stride"] * nd["cout"]
        return (nd["cin"] * es % 16 == 0 and nd["cin"] % 8 == 0 and nd["cout"] % 4 == 0 and nd["cin"] >= 32
                and m >= 32 and m % 16 == 0)
    return False


def q_bf16(x):
    return torch.from_numpy(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def q_fp8(x):
    t = torch.from_numpy(np.clip(np.asarray(x, np.float32), -448.0, 448.0))
    return t.to(torch.float8_e4m3fn).to(torch.float64).numpy()


def forward(model, weights, x, precision, act_scales=None, layer_precision=None):
    """layer_precision: optional per-layer list (one entry per conv / transposed
    conv, node order) of "fp32" / "bf16" / "fp8" overriding `precision` for the
    MFMA layers (a mixed-precision plan)."""
    params = offline.unpack_weights(model, weights)
    nodes = model["nodes"]
    outs = []
    layer = -1
    for i, nd in enumerate(nodes):
        op = nd["op"]
        if op == "input":
            outs.append(np.asarray(x, np.float64))
            continue
        if op == "add":
            outs.append(outs[nd["src"]] + outs[nd["src2"]])
            continue
        layer += 1
        w, b = params[i]
        u = offline.apply_pre(nd, outs[nd["src"]])
        lp = precision if layer_precision is None else layer_precision[layer]
        if lp != "fp32" and mfma_layer(nd, i == len(nodes) - 1, nd["src"] == 0, lp):
            if nd.get("pre_act", 0) == 1:
                # the kernel applies LeakyReLU in FP32 before rounding
                x32 = np.asarray(outs[nd["src"]], np.float32)
                u = np.where(x32 >= 0, x32, np.float32(0.2) * x32).astype(np.float64)
            if lp == "bf16":
                u = q_bf16(u)
                w = q_bf16(w)
            else:
                sa = np.float32(act_scales[layer]) / np.float32(448.0)
                qs = np.float32(1.0) / sa
                u = q_fp8(np.asarray(u, np.float32) * qs) * np.float64(sa)
                if op == "conv":      # rows = output channels
                    amax = np.max(np.abs(w.astype(np.float32)), axis=(1, 2), keepdims=True)
                else:                 # rows = (phase, output channel) of the polyphase form
                    r = nd["stride"]
                    wq = np.empty_like(w)
                    for phi in range(r):
                        taps = [phi, phi + r]
                        blk = w[:, :, taps].astype(np.float32)
                        amax = np.max(np.abs(blk), axis=(0, 2), keepdims=True)
                        s = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
                        wq[:, :, taps] = q_fp8(blk / s) * s.astype(np.float64)
                    w = wq
                if op == "conv":
                    s = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
                    w = q_fp8(w.astype(np.float32) / s) * s.astype(np.float64)
        if op == "conv":
            y = offline.conv1d(u, w, b, nd["dilation"], nd["stride"], nd["pad_l"], nd["pad_r"])
            y = offline.apply_post(nd, y)
        else:
            y = offline.conv_transpose1d(u, w, b, nd["stride"], nd["pad"])
        outs.append(y)
    return outs[-1]
