"""Model topologies as plain node lists (no arithmetic).

A model is a dict ``{"name", "nodes", "in_channels", "out_channels"}``.  Nodes
are evaluated in list order; node 0 is the input.  Node kinds:

* ``{"op": "input", "channels": C}``
* ``{"op": "conv", "src": i, "cin", "cout", "k", "dilation", "stride",
  "pad_l", "pad_r", "pre_act", "post_act"}`` -- a 1-D convolution in the
  correlation form of the paper's Eq. 1, with dilation, stride and the
  zero padding the layer was *trained* with (left ``pad_l``, right ``pad_r``).
* ``{"op": "convt", "src": i, "cin", "cout", "k", "stride", "pad",
  "pre_act"}`` -- a transposed convolution (paper Sec. 2.1) that upsamples
  time by ``stride`` and crops ``pad`` frames on each side.
* ``{"op": "add", "src": i, "src2": j}`` -- two parallel branches summed
  (paper Sec. 3.2).

``pre_act`` = 1 applies LeakyReLU(slope 0.2) to the node's input before the
convolution; ``post_act`` = 2 applies tanh to the conv output.

Weights are one flat float32 array, consumed in node order: for ``conv``
``W[cout][cin][k]`` then ``b[cout]``; for ``convt`` ``W[cin][cout][k]`` (the
PyTorch ConvTranspose1d layout) then ``b[cout]``.
"""

LRELU_SLOPE = 0.2

ACT_NONE = 0
ACT_LRELU = 1
ACT_TANH = 2


def _input(c):
    return {"op": "input", "channels": int(c)}


def _conv(src, cin, cout, k, dilation=1, stride=1, pad_l=None, pad_r=None,
          pre_act=ACT_NONE, post_act=ACT_NONE):
    if pad_l is None:
        # symmetric "same" padding of a stride-1 conv: d(k-1)/2 each side
        tot = dilation * (k - 1)
        pad_l = tot // 2
        pad_r = tot - pad_l
    return {"op": "conv", "src": int(src), "cin": int(cin), "cout": int(cout),
            "k": int(k), "dilation": int(dilation), "stride": int(stride),
            "pad_l": int(pad_l), "pad_r": int(pad_r),
            "pre_act": int(pre_act), "post_act": int(post_act)}


def _convt(src, cin, cout, ratio, pre_act=ACT_LRELU):
    # kernel 2r, symmetric crop r/2: T frames in -> T*r frames out
    assert ratio % 2 == 0, "ratio must be even for a symmetric crop"
    return {"op": "convt", "src": int(src), "cin": int(cin), "cout": int(cout),
            "k": 2 * int(ratio), "stride": int(ratio), "pad": int(ratio) // 2,
            "pre_act": int(pre_act)}


def _add(a, b):
    return {"op": "add", "src": int(a), "src2": int(b)}


def stack3():
    """Plain 3-layer cached conv stack: 1->16 (k3,d1), 16->16 (k3,d2),
    16->16 (k3,d4), symmetric padding, LeakyReLU 0.2 between layers."""
    nodes = [_input(1),
             _conv(0, 1, 16, 3, 1),
             _conv(1, 16, 16, 3, 2, pre_act=ACT_LRELU),
             _conv(2, 16, 16, 3, 4, pre_act=ACT_LRELU)]
    return {"name": "stack3", "nodes": nodes, "in_channels": 1, "out_channels": 16}


def decoder(name, latent, widths, ratios, dilations, out_k=7):
    """RAVE-style decoder: input conv k3 latent->widths[0]; per stage
    LeakyReLU -> ConvTranspose1d(stride r, k=2r) widths[s]->widths[s+1], then
    one residual block per dilation d: x + Conv_k3,d(LeakyReLU(x)); finally
    tanh(Conv_k7(LeakyReLU(x))) to one channel."""
    assert len(widths) == len(ratios) + 1
    nodes = [_input(latent), _conv(0, latent, widths[0], 3, 1)]
    for s, r in enumerate(ratios):
        cin, cout = widths[s], widths[s + 1]
        nodes.append(_convt(len(nodes) - 1, cin, cout, r))
        for d in dilations:
            x = len(nodes) - 1
            nodes.append(_conv(x, cout, cout, 3, d, pre_act=ACT_LRELU))
            nodes.append(_add(x, len(nodes) - 1))
    nodes.append(_conv(len(nodes) - 1, widths[-1], 1, out_k, 1,
                       pre_act=ACT_LRELU, post_act=ACT_TANH))
    return {"name": name, "nodes": nodes, "in_channels": latent, "out_channels": 1}


def rave_decoder_b():
    """Decoder with 16 latent channels, widths 512->256->128->64->32,
    ratios [4,4,4,2] (128 samples per latent frame), dilations 1, 3, 9."""
    return decoder("rave_b", 16, [512, 256, 128, 64, 32], [4, 4, 4, 2], [1, 3, 9])


def wide_decoder():
    """Wide decoder: 128 latent channels, widths 768->384->192->96->48,
    ratios [8,8,4,2] (512 samples per latent frame), dilations 1, 3, 9, 27."""
    return decoder("wide", 128, [768, 384, 192, 96, 48], [8, 8, 4, 2], [1, 3, 9, 27])


def strided_unit(aligned=False):
    """Cached conv then a strided conv (paper Sec. 3.1).

    ``aligned=False``: Conv k5 (right pad 2) -> Conv K=4, S=2, pads 1/1, so
    R + D_c = 3 is odd and the strided layer needs one extra delay frame.
    ``aligned=True``: Conv k3 (right pad 1) -> same strided conv, R + D_c = 2,
    no extra delay needed."""
    k0 = 3 if aligned else 5
    nodes = [_input(2),
             _conv(0, 2, 8, k0, 1),
             _conv(1, 8, 8, 4, 1, stride=2, pad_l=1, pad_r=1, pre_act=ACT_LRELU)]
    return {"name": "strided_aligned" if aligned else "strided",
            "nodes": nodes, "in_channels": 2, "out_channels": 8}


def branch_unit():
    """Two parallel convs of the same input, (k3, d1) and (k5, d2), summed
    (paper Sec. 3.2): their post-reconfiguration delays are 1 and 4 frames."""
    nodes = [_input(4),
             _conv(0, 4, 8, 3, 1),
             _conv(0, 4, 8, 5, 2),
             _add(1, 2)]
    return {"name": "branch", "nodes": nodes, "in_channels": 4, "out_channels": 8}


def branch3_unit():
    """Four parallel branches of one input, summed by three adds (Sec. 3.2,
    Eq. 3 beyond two branches): (k3, d1); (k5, d2) then (k3, d1); (k7, d3);
    and a rate excursion, a transposed conv (ratio 2) followed by a strided
    conv (K4, S2, pads 1/1) back to the input rate (Eq. 2 inside a branch).
    Post-reconfiguration delays 1, 5, 9 and 1 frames."""
    nodes = [_input(4),
             _conv(0, 4, 8, 3, 1),                                    # 1: D 1
             _conv(0, 4, 8, 5, 2),                                    # 2: D 4
             _conv(2, 8, 8, 3, 1, pre_act=ACT_LRELU),                 # 3: D 5
             _add(1, 3),                                              # 4: D 5
             _conv(0, 4, 8, 7, 3),                                    # 5: D 9
             _add(4, 5),                                              # 6: D 9
             _convt(0, 4, 8, 2, pre_act=ACT_NONE),                    # 7: rate 2, D 1
             _conv(7, 8, 8, 4, 1, stride=2, pad_l=1, pad_r=1, pre_act=ACT_LRELU),   # 8: rate 1, D 1
             _add(6, 8)]                                              # 9: D 9
    return {"name": "branch3", "nodes": nodes, "in_channels": 4, "out_channels": 8}


def encoder(name="encoder", ratios=(4, 4, 4, 2), widths=(16, 32, 64, 128, 256), latent=16):
    """RAVE-style strided-conv encoder: Conv k7 1->widths[0], then per ratio
    r: LeakyReLU -> Conv(k=2r+1, stride r, pads r/r), then LeakyReLU -> Conv k3
    to the latent size.  Input buffers must be multiples of prod(ratios)."""
    nodes = [_input(1), _conv(0, 1, widths[0], 7, 1)]
    for s, r in enumerate(ratios):
        nodes.append(_conv(len(nodes) - 1, widths[s], widths[s + 1], 2 * r + 1, 1,
                           stride=r, pad_l=r, pad_r=r, pre_act=ACT_LRELU))
    nodes.append(_conv(len(nodes) - 1, widths[len(ratios)], latent, 3, 1, pre_act=ACT_LRELU))
    return {"name": name, "nodes": nodes, "in_channels": 1, "out_channels": latent}


def autoencoder():
    """Audio in, audio out: the strided encoder (ratios 4,4,4,2 to 16 latent
    channels) feeding the rave_b decoder (ratios 4,4,4,2 back to one channel);
    input buffers are multiples of 128 samples."""
    enc, dec = encoder(), rave_decoder_b()
    base = len(enc["nodes"]) - 1   # the decoder's input is the encoder's output
    nodes = [dict(n) for n in enc["nodes"]]
    for n in dec["nodes"][1:]:
        n = dict(n)
        for key in ("src", "src2"):
            if key in n:
                n[key] = n[key] + base
        nodes.append(n)
    return {"name": "autoencoder", "nodes": nodes, "in_channels": 1, "out_channels": 1}


def outconv_unit():
    """Input conv 8->64 (k3), a transposed conv 64->32 (ratio 32), one residual
    block x + Conv_k3,d3(LeakyReLU(x)) at 32 channels, then a one-channel
    output conv with dilation and no tanh: Conv_k5,d3(LeakyReLU(x)), padding
    6/6."""
    nodes = [_input(8),
             _conv(0, 8, 64, 3, 1),
             _convt(1, 64, 32, 32),
             _conv(2, 32, 32, 3, 3, pre_act=ACT_LRELU),
             _add(2, 3),
             _conv(4, 32, 1, 5, 3, pre_act=ACT_LRELU)]
    return {"name": "outconv", "nodes": nodes, "in_channels": 8, "out_channels": 1}


def outconv64_unit():
    """Input conv 8->64 (k3), a transposed conv 64->64 (ratio 10), one residual
    block x + Conv_k3,d1(LeakyReLU(x)) at 64 channels, then a one-channel
    output conv Conv_k5,d3(LeakyReLU(x)) (padding 6/6) whose 12-frame cache is
    longer than the 10 frames a 1-frame buffer brings it."""
    nodes = [_input(8),
             _conv(0, 8, 64, 3, 1),
             _convt(1, 64, 64, 10),
             _conv(2, 64, 64, 3, 1, pre_act=ACT_LRELU),
             _add(2, 3),
             _conv(4, 64, 1, 5, 3, pre_act=ACT_LRELU)]
    return {"name": "outconv64", "nodes": nodes, "in_channels": 8, "out_channels": 1}


def outconv48_unit():
    """Input conv 8->64 (k3), a transposed conv 64->48 (ratio 10), one residual
    block x + Conv_k3,d3(LeakyReLU(x)) at 48 channels (a 64-row tile of which
    16 rows are padding), then the decoder's output conv
    tanh(Conv_k7(LeakyReLU(x))) to one channel."""
    nodes = [_input(8),
             _conv(0, 8, 64, 3, 1),
             _convt(1, 64, 48, 10),
             _conv(2, 48, 48, 3, 3, pre_act=ACT_LRELU),
             _add(2, 3),
             _conv(4, 48, 1, 7, 1, pre_act=ACT_LRELU, post_act=ACT_TANH)]
    return {"name": "outconv48", "nodes": nodes, "in_channels": 8, "out_channels": 1}


def pair48_unit():
    """Input conv 8->64 (k3), a transposed conv 64->48 (ratio 32), two residual
    blocks x + Conv_k3,d(LeakyReLU(x)) at 48 channels (d = 1 then 3: a pair of
    residual convs on a 64-row tile with 16 padding rows), then the decoder's
    output conv tanh(Conv_k7(LeakyReLU(x))) to one channel."""
    nodes = [_input(8),
             _conv(0, 8, 64, 3, 1),
             _convt(1, 64, 48, 32),
             _conv(2, 48, 48, 3, 1, pre_act=ACT_LRELU),
             _add(2, 3),
             _conv(4, 48, 48, 3, 3, pre_act=ACT_LRELU),
             _add(4, 5),
             _conv(6, 48, 1, 7, 1, pre_act=ACT_LRELU, post_act=ACT_TANH)]
    return {"name": "pair48", "nodes": nodes, "in_channels": 8, "out_channels": 1}


def model_by_name(name):
    table = {"stack3": stack3, "rave_b": rave_decoder_b, "wide": wide_decoder, "outconv": outconv_unit,
             "autoencoder": autoencoder, "outconv64": outconv64_unit, "outconv48": outconv48_unit, "pair48": pair48_unit,
             "strided": lambda: strided_unit(False),
             "strided_aligned": lambda: strided_unit(True),
             "branch": branch_unit, "branch3": branch3_unit, "encoder": encoder}
    return table[name]()


# Mixed-precision plans: the layers (indices among the conv / transposed-conv
# nodes, node order) whose operands are FP8 e4m3; every other layer runs on
# BF16.  e4m3 keeps three mantissa bits, and one rounding of the weights and
# activations of a full-width layer costs ~28 dB of SNR (~34 dB for a residual
# branch, whose output is half the size of the stream it is added to); these
# errors add up over the layers in series, so an all-FP8 decoder stays near
# 19 dB.  The plans below are the two-layer sets with the most FLOPs that keep
# the decoder above 30 dB against the FP64 offline model with margin (a third
# layer brings it to ~30.0 dB).  tests/golden/fp8_plans.py re-derives them
# from a rounding emulation of the offline model.
FP8_LAYERS = {
    # rave_b: the stage-1 residual convs with dilation 1 and 3 (256 channels)
    "rave_b": (2, 3),
    # wide: the stage-3 residual convs with dilation 3 and 27 (96 channels)
    "wide": (13, 15),
}


def fp8_plan(model):
    """Per-layer precision list ("fp8" / "bf16", one per conv / transposed
    conv in node order) of the mixed FP8 plan of a decoder model."""
    layers = [nd for nd in model["nodes"] if nd["op"] in ("conv", "convt")]
    fp8 = set(FP8_LAYERS[model["name"]])
    return ["fp8" if i in fp8 else "bf16" for i in range(len(layers))]


def n_weights(model):
    """Number of float32 values in the flat weight array of ``model``."""
    n = 0
    for nd in model["nodes"]:
        if nd["op"] == "conv":
            n += nd["cout"] * nd["cin"] * nd["k"] + nd["cout"]
        elif nd["op"] == "convt":
            n += nd["cin"] * nd["cout"] * nd["k"] + nd["cout"]
    return n
