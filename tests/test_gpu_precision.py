"""GPU checks of the MFMA paths (FP32, BF16, FP8 e4m3) against the FP64
oracle (max-abs / SNR over the comparison window) and against a CPU
emulation of the intended operand rounding; multi-stream workloads at the
benchmark configurations' sizes with the oracle on sampled streams."""
import numpy as np
import pytest

import scgen
from oracle import metrics, offline
from gpu_helpers import log, oracle_compare, run_stream, weights_for
import emulate

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_SNR = 40.0
FP8_SNR = 30.0


def _sc():
    import paper_2204_07064_amd as sc
    return sc


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _model(sc, m, w, prec, scales, options=0):
    """prec "mix": the model's mixed FP8 plan (FP8 layers of scgen.fp8_plan,
    the others on BF16)."""
    if prec == "mix":
        return sc.Model(m, w, act_scales=scales, options=options, layer_precision=scgen.fp8_plan(m))
    return sc.Model(m, w, prec, act_scales=scales if prec == "fp8" else None, options=options)


def _fp8_scales(sc, m, w, channels):
    from paper_2204_07064_amd import calibrate
    cal = [scgen.latents(channels, 64, 1 + i) for i in range(4)]
    return calibrate.act_scales(sc, m, w, cal)


@pytest.mark.parametrize("name", ["rave_b", "wide"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "mix"])
def test_operand_twins_bitwise(name, prec):
    """MFMA layers reading the operand copy written by their producer give
    bitwise the same stream as layers that activate and round on load."""
    sc = _sc()
    m, w = weights_for(name)
    c = m["in_channels"]
    scales = _fp8_scales(sc, m, w, c) if prec in ("fp8", "mix") else None
    x = scgen.stream_latents(c, 40, 2)
    splits = [1, 3, 16, 8, 12]
    a = run_stream(_model(sc, m, w, prec, scales), x, splits)
    b = run_stream(_model(sc, m, w, prec, scales, options=4), x, splits)
    assert np.array_equal(a, b)
    if prec == "mix":       # split invariance of the mixed plan
        assert np.array_equal(a, run_stream(_model(sc, m, w, prec, scales), x, [20, 20]))


def _batched_streams(sc, mod, xs, lens):
    """Steps of len(xs) streams; step j gives stream i lens[i][j] frames.
    Returns each stream's concatenated output (numpy float64)."""
    streams = [sc.Stream(mod, int(max(l))) for l in lens]
    xd = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda() for x in xs]
    pos = [0] * len(xs)
    outs = [[] for _ in xs]
    for j in range(len(lens[0])):
        ins = []
        for i in range(len(xs)):
            n = int(lens[i][j])
            ins.append(xd[i][:, pos[i]:pos[i] + n].contiguous())
            pos[i] += n
        for i, o in enumerate(sc.process_batch(mod, streams, ins)):
            outs[i].append(o)
    torch.cuda.synchronize()
    return [torch.cat(o, dim=1).cpu().double().numpy() for o in outs]


@pytest.mark.parametrize("name", ["rave_b", "wide"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8", "mix"])
def test_window_kernel_bitwise(name, prec):
    """Narrow stride-1 MFMA convs that stage each tile's [cache | new frames]
    window in LDS give bitwise the same streams as the chunk-gathering kernel,
    in a batch whose tiles span several streams of uneven buffers."""
    sc = _sc()
    m, w = weights_for(name)
    c = m["in_channels"]
    scales = _fp8_scales(sc, m, w, c) if prec in ("fp8", "mix") else None
    rng = np.random.default_rng(5)
    n_str, n_steps = (9, 4) if name == "rave_b" else (5, 3)
    lens = [[int(v) for v in rng.choice([1, 2, 3, 5, 8], size=n_steps)] for _ in range(n_str)]
    xs = [scgen.stream_latents(c, sum(l), 30 + i) for i, l in enumerate(lens)]
    # the output conv on its own launch in both (the gathering kernel has no
    # fused form of it)
    nof = sc._native.SC_MODEL_NO_OUT_FUSION
    win = _model(sc, m, w, prec, scales, options=nof)
    win.profile(True)
    a = _batched_streams(sc, win, xs, lens)
    impls = {p["node"]: p["impl"] for p in win.profile_read()}
    win.profile(False)
    assert 2 in impls.values(), impls          # the window kernel ran
    b = _batched_streams(sc, _model(sc, m, w, prec, scales, options=8 | nof), xs, lens)
    for i in range(n_str):
        assert np.array_equal(a[i], b[i]), i


@pytest.mark.parametrize("prec,split", [("bf16", True), ("bf16", False), ("fp8", True), ("mix", False)])
def test_convt_window_fusion_bitwise(prec, split):
    """The narrow stages' transposed conv computed inside the launch of the
    residual conv after it gives bitwise the same streams as its own launch,
    in steps of many streams of uneven buffers (1-frame buffers included),
    split into concurrent halves or not."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16) if prec in ("fp8", "mix") else None
    rng = np.random.default_rng(13)
    lens = [[int(v) for v in rng.choice([1, 2, 4, 8, 16, 32], size=3)] for _ in range(96)]
    xs = [scgen.stream_latents(16, sum(l), 700 + i) for i, l in enumerate(lens)]
    base = 0 if split else sc._native.SC_MODEL_NO_SPLIT
    fused = _model(sc, m, w, prec, scales, options=base)
    fused.profile(True)
    a = _batched_streams(sc, fused, xs, lens)
    convt = {p["node"]: p["launches"] for p in fused.profile_read() if p["kind"] == 2}
    fused.profile(False)
    log("convt fusion %s split=%s launches per transposed conv: %s" % (prec, split, convt))
    if prec != "mix":       # computed inside the next launch (the 32-channel stage)
        assert sum(v == 0 for v in convt.values()) >= 1, convt
    b = _batched_streams(sc, _model(sc, m, w, prec, scales, options=base | sc._native.SC_MODEL_NO_CONVT_FUSION),
                         xs, lens)
    for i in range(len(lens)):
        assert np.array_equal(a[i], b[i]), i


@pytest.mark.parametrize("prec,split", [("fp32", True), ("bf16", False), ("bf16", True), ("fp8", True)])
def test_direct_input_bitwise(prec, split):
    """The input conv gathering the latents straight from the callers'
    channel-major buffers (no packing launch) gives bitwise the same streams
    as packing them first, in steps of many streams of uneven buffers (1-frame
    buffers included), split or not, and with the warm-up mask."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16) if prec == "fp8" else None
    rng = np.random.default_rng(17)
    lens = [[int(v) for v in rng.choice([1, 2, 3, 8, 16, 32], size=3)] for _ in range(72)]
    xs = [scgen.stream_latents(16, sum(l), 900 + i) for i, l in enumerate(lens)]
    base = 0 if split else sc._native.SC_MODEL_NO_SPLIT
    a = _batched_streams(sc, _model(sc, m, w, prec, scales, options=base), xs, lens)
    b = _batched_streams(sc, _model(sc, m, w, prec, scales, options=base | sc._native.SC_MODEL_NO_INPUT_DIRECT),
                         xs, lens)
    for i in range(len(lens)):
        assert np.array_equal(a[i], b[i]), i
    # one stream with the warm-up mask, buffer by buffer
    x = scgen.stream_latents(16, 40, 5)
    outs = []
    for opt in (base, base | sc._native.SC_MODEL_NO_INPUT_DIRECT):
        mod = _model(sc, m, w, prec, scales, options=opt)
        outs.append(run_stream(mod, x, [1, 7, 32], stream=sc.Stream(mod, 32, warmup_mask=True)))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("prec,split", [("bf16", False), ("bf16", True), ("fp8", True), ("mix", False)])
def test_conv_pair_fusion_bitwise(prec, split):
    """Two residual window convs of the 64-channel stage in one launch (the
    first one's output computed per tile and never written) give bitwise the
    same streams as two launches: steps of many streams of uneven buffers
    (1-frame buffers included), split into concurrent halves or not, and one
    stream with the warm-up mask buffer by buffer; the caches the pair writes
    carry the next step."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16) if prec in ("fp8", "mix") else None
    rng = np.random.default_rng(19)
    lens = [[int(v) for v in rng.choice([1, 2, 4, 8, 16, 32], size=4)] for _ in range(80)]
    xs = [scgen.stream_latents(16, sum(l), 1100 + i) for i, l in enumerate(lens)]
    base = 0 if split else sc._native.SC_MODEL_NO_SPLIT
    fused = _model(sc, m, w, prec, scales, options=base)
    fused.profile(True)
    a = _batched_streams(sc, fused, xs, lens)
    idle = [p["node"] for p in fused.profile_read() if p["kind"] == 1 and p["launches"] == 0]
    fused.profile(False)
    log("pair fusion %s split=%s conv nodes computed inside the next launch: %s" % (prec, split, idle))
    assert len(idle) == 2, idle       # the first conv of each fused pair (64- and 32-channel stages)
    with pytest.raises(sc._native.ScError):   # the first conv's output is never formed
        fused.enable_amax(True)
    b = _batched_streams(sc, _model(sc, m, w, prec, scales, options=base | sc._native.SC_MODEL_NO_PAIR_FUSION),
                         xs, lens)
    for i in range(len(lens)):
        assert np.array_equal(a[i], b[i]), i
    x = scgen.stream_latents(16, 40, 6)
    outs = []
    for opt in (base, base | sc._native.SC_MODEL_NO_PAIR_FUSION):
        mod = _model(sc, m, w, prec, scales, options=opt)
        outs.append(run_stream(mod, x, [1, 7, 32], stream=sc.Stream(mod, 32, warmup_mask=True)))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("name,prec", [("pair48", "bf16"), ("pair48", "fp8"), ("wide", "bf16")])
def test_conv_pair_48_channels_bitwise(name, prec):
    """The residual pair on a 64-row tile with 48 channels (16 padding rows;
    the unit model's second conv also computes the output conv) gives bitwise
    the same streams as two launches: many streams of uneven buffers, split
    and unsplit steps, state carried across steps."""
    sc = _sc()
    m, w = weights_for(name)
    c = m["in_channels"]
    scales = _fp8_scales(sc, m, w, c) if prec == "fp8" else None
    rng = np.random.default_rng(23)
    n_str = 40 if name == "wide" else 64
    choices = [1, 2, 3, 5, 8] if name == "wide" else [1, 2, 4, 8, 16, 32]
    lens = [[int(v) for v in rng.choice(choices, size=3)] for _ in range(n_str)]
    xs = [scgen.stream_latents(c, sum(l), 1300 + i) for i, l in enumerate(lens)]
    for base in (0, sc._native.SC_MODEL_NO_SPLIT):
        fused = _model(sc, m, w, prec, scales, options=base)
        fused.profile(True)
        a = _batched_streams(sc, fused, xs, lens)
        idle = [p["node"] for p in fused.profile_read() if p["kind"] == 1 and p["launches"] == 0]
        fused.profile(False)
        log("48-channel pair %s %s options=%d: conv nodes inside the next launch: %s" % (name, prec, base, idle))
        assert len(idle) == 1, idle
        b = _batched_streams(sc, _model(sc, m, w, prec, scales, options=base | sc._native.SC_MODEL_NO_PAIR_FUSION),
                             xs, lens)
        for i in range(n_str):
            assert np.array_equal(a[i], b[i]), (base, i)


def test_mfma_fp32_matches_wavefront_fp32():
    """The FP32 MFMA path (input conv included) and the FP32 wavefront path
    sum in different orders; each is pinned to the FP64 oracle at 1e-5 by the
    parity tests, and they agree to a few ulps per layer (bound 4e-6 over the
    18 layers)."""
    sc = _sc()
    m, w = weights_for("rave_b")
    x = scgen.stream_latents(16, 64, 1)
    a = run_stream(sc.Model(m, w, "fp32"), x, [16] * 4)
    b = run_stream(sc.Model(m, w, "fp32", options=2), x, [16] * 4)
    log("mfma vs valu fp32 max-abs %.3e" % np.max(np.abs(a - b)))
    assert np.max(np.abs(a - b)) <= 4e-6


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_single_stream_precision(prec):
    """Whole decoder, one stream, 16 buffers of 16 frames, against the oracle.
    (Network-level comparison with the rounding emulation is loose by nature:
    the FP32 accumulation already changes a few rounding decisions, and those
    cascade through the 16 rounded layers -- the per-layer test below is the
    tight one.)"""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16) if prec == "fp8" else None
    plan = scgen.fp8_plan(m) if prec == "fp8" else None
    mod = sc.Model(m, w, prec, act_scales=scales, layer_precision=plan)
    x = scgen.stream_latents(16, 256, 0)
    s = run_stream(mod, x, [16] * 16)
    err, snr, y = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    ye = emulate.forward(m, w, x, prec, scales, plan)
    sw, ew = metrics.aligned(s, ye, mod.latency, mod.warmup)
    log("%s: vs oracle max-abs %.3e SNR %.2f dB; vs rounding emulation SNR %.1f dB"
        % (prec, err, snr, metrics.snr_db(sw, ew)))
    if prec == "bf16":
        assert snr >= BF16_SNR
    else:
        assert snr >= FP8_SNR        # the mixed plan (scgen.fp8_plan)


def test_autoencoder_bf16_snr():
    """Audio in, audio out (strided encoder feeding the decoder), BF16, one
    stream of white noise in 128-sample multiples, against the FP64 oracle: the
    encoder's strided and narrow layers run in FP32, the decoder's wide layers
    on BF16 operands, so the BF16 SNR target applies to the whole path."""
    sc = _sc()
    m, w = weights_for("autoencoder")
    mod = sc.Model(m, w, "bf16")
    x = scgen.stream_latents(1, 128 * 48, 3)
    s = run_stream(mod, x, [128 * k for k in (1, 4, 16, 2, 8, 1, 16)])
    err, snr, _ = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    log("autoencoder bf16: vs oracle max-abs %.3e SNR %.2f dB" % (err, snr))
    assert snr >= BF16_SNR


def _one_layer_model(kind, c_in, c_out, dil=3, ratio=4):
    """identity k1 conv (FP32 wavefront, exact copy) -> layer under test (MFMA)
    -> identity k1 conv to the output (exact copy)."""
    nodes = [{"op": "input", "channels": c_in},
             {"op": "conv", "src": 0, "cin": c_in, "cout": c_in, "k": 1, "dilation": 1, "stride": 1,
              "pad_l": 0, "pad_r": 0, "pre_act": 0, "post_act": 0}]
    if kind == "residual":
        nodes.append({"op": "conv", "src": 1, "cin": c_in, "cout": c_in, "k": 3, "dilation": dil, "stride": 1,
                      "pad_l": dil, "pad_r": dil, "pre_act": 1, "post_act": 0})
        nodes.append({"op": "add", "src": 1, "src2": 2})
        c_last = c_in
    elif kind == "conv":
        nodes.append({"op": "conv", "src": 1, "cin": c_in, "cout": c_out, "k": 3, "dilation": dil, "stride": 1,
                      "pad_l": dil, "pad_r": dil, "pre_act": 1, "post_act": 0})
        c_last = c_out
    else:
        nodes.append({"op": "convt", "src": 1, "cin": c_in, "cout": c_out, "k": 2 * ratio, "stride": ratio,
                      "pad": ratio // 2, "pre_act": 1})
        c_last = c_out
    nodes.append({"op": "conv", "src": len(nodes) - 1, "cin": c_last, "cout": c_last, "k": 1, "dilation": 1,
                  "stride": 1, "pad_l": 0, "pad_r": 0, "pre_act": 0, "post_act": 0})
    m = {"name": "one_" + kind, "nodes": nodes, "in_channels": c_in, "out_channels": c_last}
    rng = np.random.default_rng(11)
    parts = []
    for nd in nodes:
        if nd["op"] not in ("conv", "convt"):
            continue
        if nd["k"] == 1:
            parts += [np.eye(nd["cout"], dtype=np.float32).reshape(-1), np.zeros(nd["cout"], np.float32)]
        else:
            shape = (nd["cout"], nd["cin"], nd["k"]) if nd["op"] == "conv" else (nd["cin"], nd["cout"], nd["k"])
            parts += [(rng.uniform(-1, 1, size=shape) / np.sqrt(nd["cin"] * 2)).astype(np.float32).ravel(),
                      rng.uniform(-0.1, 0.1, size=nd["cout"]).astype(np.float32)]
    return m, np.concatenate(parts)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("kind,c_in,c_out", [("residual", 64, 64), ("conv", 96, 128), ("convt", 128, 32),
                                             ("convt", 64, 48)])
def test_mfma_layer_rounding(prec, kind, c_in, c_out):
    """One MFMA layer, streamed in uneven buffers (cache / carry paths) with
    the warm-up mask: equals the offline layer evaluated in FP64 on the same
    rounded operands up to FP32 accumulation (relative 1e-5)."""
    sc = _sc()
    m, w = _one_layer_model(kind, c_in, c_out)
    layer_scales = np.full(3, 3.0, np.float32)
    mod = sc.Model(m, w, prec, act_scales=layer_scales if prec == "fp8" else None)
    frames = 200
    x = scgen.stream_latents(c_in, frames, 9)
    s = run_stream(mod, x, [1, 7, 32, 3, 64, 5, 88], warmup_mask=True)
    ye = emulate.forward(m, w, x, prec, layer_scales)
    D = mod.latency
    err = np.max(np.abs(s[:, D:] - ye[:, :ye.shape[1] - D]))
    ref = np.max(np.abs(ye))
    log("%s %s %d->%d: max-abs vs rounding emulation %.3e (|y|max %.2f)" % (prec, kind, c_in, c_out, err, ref))
    assert np.all(s[:, :D] == 0)
    # FP32 / BF16 MFMA: FP32 accumulation, 1e-5.  The FP8 f8f6f4 MFMA was
    # measured at up to 2.5e-5 relative on identical operands (its internal
    # accumulation is coarser than FP32); one mis-rounded FP8 operand would
    # cost ~1e-3, so 1e-4 still pins the rounding.
    tol = 1e-4 if prec == "fp8" else 1e-5
    assert err <= tol * ref


def test_fp8_snr_target():
    """The decoder with its mixed FP8 plan (the FP8 layers of scgen.fp8_plan,
    every other wide layer on BF16; FP32 state and accumulation) meets the
    30 dB SNR target against the FP64 oracle on uneven buffers, and its
    result equals the rounding emulation of the same plan far above that."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16)
    plan = scgen.fp8_plan(m)
    mod = sc.Model(m, w, act_scales=scales, layer_precision=plan)
    assert mod.precision == "fp8"
    x = scgen.stream_latents(16, 128, 0)
    s = run_stream(mod, x, [16, 1, 31, 8, 8, 3, 29, 16, 16])
    err, snr, _ = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    ye = emulate.forward(m, w, x, "fp8", scales, plan)
    sw, ew = metrics.aligned(s, ye, mod.latency, mod.warmup)
    log("fp8 plan %s: vs oracle max-abs %.3e SNR %.2f dB; vs emulation %.1f dB"
        % ([i for i, p in enumerate(plan) if p == "fp8"], err, snr, metrics.snr_db(sw, ew)))
    assert snr >= FP8_SNR
    assert metrics.snr_db(sw, ew) >= 45.0


def test_fp8_all_layers_is_format_limited():
    """Every wide layer on FP8 e4m3 (no mixed plan): the GPU result tracks
    the CPU emulation of that rounding (so the kernels round as intended) and
    both sit near 19 dB against the FP64 oracle -- e4m3's three mantissa bits
    cost ~28 dB per full-width layer, and 16 layers in series add up.  This
    is the measured reason for the mixed plan; the 30 dB target is not
    claimed for this configuration."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = _fp8_scales(sc, m, w, 16)
    mod = sc.Model(m, w, "fp8", act_scales=scales)
    x = scgen.stream_latents(16, 128, 0)
    s = run_stream(mod, x, [16] * 8)
    _, snr, y = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    ye = emulate.forward(m, w, x, "fp8", scales)
    lo, hi = metrics.window(mod.latency, mod.warmup, y.shape[-1])
    snr_emul = metrics.snr_db(ye[..., lo:hi], y[..., lo:hi])
    log("all-FP8 decoder: GPU %.2f dB, emulation %.2f dB vs oracle" % (snr, snr_emul))
    assert abs(snr - snr_emul) <= 1.5
    assert snr < FP8_SNR


def _batched(sc, mod, xs, lens_per_step):
    """Run len(xs) streams in batched steps; lens_per_step[k][i] frames for
    stream i at step k.  Returns the concatenated outputs (numpy float64)."""
    streams = [sc.Stream(mod, int(max(l[i] for l in lens_per_step))) for i in range(len(xs))]
    xd = [torch.from_numpy(x).cuda() for x in xs]
    pos = [0] * len(xs)
    outs = [[] for _ in xs]
    for lens in lens_per_step:
        ins = []
        for i, n in enumerate(lens):
            ins.append(xd[i][:, pos[i]:pos[i] + n].contiguous())
            pos[i] += n
        ys = sc.process_batch(mod, streams, ins)
        for i, y in enumerate(ys):
            outs[i].append(y)
    torch.cuda.synchronize()
    return [torch.cat(o, dim=1).cpu().double().numpy() for o in outs]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_64_streams_1024_frames(prec):
    """64 concurrent streams x 1024 latent frames, 16-frame buffers: the
    oracle on 3 sampled streams (whole signals), the rest by invariance."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    n_s, frames, buf = 64, 1024, 16
    xs = [scgen.stream_latents(16, frames, i) for i in range(n_s)]
    outs = _batched(sc, mod, xs, [[buf] * n_s for _ in range(frames // buf)])
    pooled_s, pooled_y, worst = [], [], 1e9
    for i in (0, 31, 63):
        y = offline.forward(m, w, xs[i])
        sw, yw = metrics.aligned(outs[i], y, mod.latency, mod.warmup)
        pooled_s.append(sw)
        pooled_y.append(yw)
        e = metrics.max_abs(sw, yw)
        worst = min(worst, metrics.snr_db(sw, yw))
        log("%s stream %d: max-abs %.3e snr %.2f dB" % (prec, i, e, metrics.snr_db(sw, yw)))
        if prec == "fp32":
            assert e <= FP32_TOL
    snr = metrics.snr_db(np.concatenate(pooled_s), np.concatenate(pooled_y))
    log("%s pooled SNR %.2f dB (min per stream %.2f)" % (prec, snr, worst))
    if prec == "bf16":
        assert snr >= BF16_SNR
    # stream 5 alone in a different split equals its batched result bitwise
    alone = run_stream(mod, xs[5], scgen.random_split(frames, 3, 32))
    assert np.array_equal(alone, outs[5])


def test_serving_mix_uneven_buffers_bf16():
    """256 streams, buffer lengths uniform over {1,2,4,8,16,32} per step;
    sampled streams against the oracle; one stream alone vs in the mix."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "bf16")
    n_s, steps = 256, 6
    lens = [scgen.buffer_lengths(steps, (1, 2, 4, 8, 16, 32), 7 * 100003 + i) for i in range(n_s)]
    frames = [sum(l) for l in lens]
    xs = [scgen.stream_latents(16, frames[i], i) for i in range(n_s)]
    outs = _batched(sc, mod, xs, [[lens[i][k] for i in range(n_s)] for k in range(steps)])
    for i in (0, 100, 255):
        y = offline.forward(m, w, xs[i])
        sw, yw = metrics.aligned(outs[i], y, mod.latency, mod.warmup)
        if sw.size:
            log("mix stream %d (%d frames): snr %.2f dB" % (i, frames[i], metrics.snr_db(sw, yw)))
            assert metrics.snr_db(sw, yw) >= BF16_SNR
    alone = run_stream(mod, xs[100], lens[100])
    assert np.array_equal(alone, outs[100])


def test_wide_decoder_1024_streams():
    """Wide decoder (128 latents, 768->...->48, ratios 8,8,4,2, dilations up
    to 27): 1024 streams with uneven 1..8-frame buffers, in FP32, BF16 and the
    mixed FP8 plan; oracle on sampled streams (FP32 max-abs per stream, BF16
    and FP8 pooled SNR)."""
    sc = _sc()
    m, w = weights_for("wide")
    scales = _fp8_scales(sc, m, w, 128)
    n_s, steps = 1024, 10
    lens = [scgen.buffer_lengths(steps, range(1, 9), 5 * 100003 + i) for i in range(n_s)]
    frames = [sum(l) for l in lens]
    xs = [scgen.stream_latents(128, frames[i], i) for i in range(n_s)]
    res = {}
    ys = {i: offline.forward(m, w, xs[i]) for i in (3, 700, 1023)}
    for prec in ("fp8", "bf16", "fp32"):
        plan = scgen.fp8_plan(m) if prec == "fp8" else None
        mod = sc.Model(m, w, prec, act_scales=scales if prec == "fp8" else None, layer_precision=plan)
        outs = _batched(sc, mod, xs, [[lens[i][k] for i in range(n_s)] for k in range(steps)])
        ss, yy = [], []
        for i, y in ys.items():
            sw, yw = metrics.aligned(outs[i], y, mod.latency, mod.warmup)
            assert sw.size > 0
            if prec == "fp32":
                e = metrics.max_abs(sw, yw)
                log("wide fp32 stream %d: max-abs %.3e" % (i, e))
                assert e <= FP32_TOL
            ss.append(sw)
            yy.append(yw)
        res[prec] = metrics.snr_db(np.concatenate(ss, axis=1), np.concatenate(yy, axis=1))
        mod.close()
    log("wide decoder pooled SNR: %s" % res)
    assert res["bf16"] >= BF16_SNR
    assert res["fp8"] >= FP8_SNR
