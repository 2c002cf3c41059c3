"""GPU parity of the streaming library against the FP64 oracle (FP32 path),
and the method's invariants on the device: the streamed output equals the
offline output delayed by the latency (paper Sec. 4.2), bitwise independent of
the buffer split, of batching with other streams, and of reset."""
import numpy as np
import pytest

import scgen
from oracle import metrics
from gpu_helpers import log, oracle_compare, run_stream, weights_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def _sc():
    import paper_2204_07064_amd as sc
    return sc


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,frames,buf,options", [
    ("stack3", 16384, 512, 0),          # 3-layer stack, 32 buffers of 512
    ("rave_b", 256, 16, 0),             # decoder, 16 buffers of 16 latent frames
    ("rave_b", 40, 1, 0),               # 1-frame buffers, below the receptive field
    ("rave_b", 96, 16, 2),              # every layer on the FP32 wavefront kernels
    ("rave_b", 64, 9, 1),               # residual sums as explicit delay lines
    ("strided", 256, 8, 0),             # Eq. 2 alignment delay D_a = 1
    ("strided_aligned", 256, 6, 0),
    ("branch", 300, 7, 0),              # Eq. 3 branch delays (3, 0)
    ("branch3", 301, 5, 0),             # four branches, three adds, a rate excursion
    ("encoder", 128 * 40, 128 * 3, 0),  # strided encoder, buffers multiple of 128
    ("autoencoder", 128 * 24, 128 * 3, 0),  # strided encoder feeding the decoder, audio in and out
    ("outconv", 96, 3, 0),              # output conv (k5, d3, no tanh) fused into a window conv
    ("outconv", 96, 3, 32),             # the same as its own launch
    ("outconv64", 60, 1, 0),            # 64-channel fused form; 10-frame buffers, 12-frame cache
    ("outconv64", 97, 3, 0),
    ("outconv48", 64, 1, 0),            # 48 channels on a 64-row tile (16 padding rows), tanh, k7
    ("outconv48", 97, 3, 0),
    ("pair48", 61, 2, 0),
])
def test_fp32_parity(name, frames, buf, options):
    sc = _sc()
    log("parity %s frames=%d buf=%d options=%d" % (name, frames, buf, options))
    m, w = weights_for(name)
    x = scgen.stream_latents(m["in_channels"], frames, 0)
    mod = sc.Model(m, w, "fp32", options=options)
    splits = scgen.split_lengths(frames, buf)
    s = run_stream(mod, x, splits)
    err, snr, _ = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    log("  max-abs %.3e snr %.1f dB" % (err, snr))
    assert err <= FP32_TOL


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_long_buffers(prec):
    """Long buffers of one stream (1024 and 1000 latent frames: 131072 output
    samples in one buffer, window tiles and MFMA column tiles all inside one
    stream, a ragged last tile) match the oracle, and equal the same input
    streamed in short buffers bitwise."""
    sc = _sc()
    m, w = weights_for("rave_b")
    x = scgen.stream_latents(16, 2024, 11)
    mod = sc.Model(m, w, prec)
    s = run_stream(mod, x, [1024, 1000])
    if prec == "fp32":
        err, snr, _ = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
        log("  long buffers: max-abs %.3e snr %.1f dB" % (err, snr))
        assert err <= FP32_TOL
    short = run_stream(mod, x, scgen.split_lengths(2024, 8))
    assert np.array_equal(s, short)


def test_split_invariance_bitwise():
    sc = _sc()
    m, w = weights_for("rave_b")
    x = scgen.stream_latents(16, 64, 3)
    mod = sc.Model(m, w, "fp32")
    ref = run_stream(mod, x, [64])
    for seed in range(3):
        s = run_stream(mod, x, scgen.random_split(64, seed, 12))
        assert np.array_equal(s, ref)


def test_fusion_is_bitwise_equal_to_delay_lines():
    sc = _sc()
    m, w = weights_for("rave_b")
    x = scgen.stream_latents(16, 48, 4)
    # (the output conv runs on its own in both: with explicit delay lines the
    # conv before it is no window conv to fuse it into)
    nof = sc._native.SC_MODEL_NO_OUT_FUSION
    a = run_stream(sc.Model(m, w, "fp32", options=nof), x, [5, 11, 32])
    b = run_stream(sc.Model(m, w, "fp32", options=1 | nof), x, [5, 11, 32])
    assert np.array_equal(a, b)


def test_warmup_mask():
    sc = _sc()
    m, w = weights_for("rave_b")
    x = scgen.stream_latents(16, 48, 5)
    mod = sc.Model(m, w, "fp32")
    s = run_stream(mod, x, [7, 9, 32], warmup_mask=True)
    D = mod.latency
    assert np.all(s[:, :D] == 0.0)
    err, _, _ = oracle_compare(m, w, x, s, D, 0)
    assert err <= FP32_TOL


def test_reset_equals_fresh():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    x = scgen.stream_latents(16, 32, 6)
    st = sc.Stream(mod, 32)
    run_stream(mod, scgen.stream_latents(16, 13, 7), [13], stream=st)
    st.reset()
    assert st.position == 0
    a = run_stream(mod, x, [10, 22], stream=st)
    b = run_stream(mod, x, [10, 22])
    assert np.array_equal(a, b)


def test_batch_equals_alone_bitwise():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    lens = [1, 4, 16, 2, 32, 8, 3]
    xs = [scgen.stream_latents(16, 3 * n, 20 + i) for i, n in enumerate(lens)]
    alone = [run_stream(mod, x, [n, n, n]) for x, n in zip(xs, lens)]
    streams = [sc.Stream(mod, 32) for _ in lens]
    outs = [[] for _ in lens]
    for step in range(3):
        xd = [torch.from_numpy(x[:, step * n:(step + 1) * n].copy()).cuda() for x, n in zip(xs, lens)]
        ys = sc.process_batch(mod, streams, xd)
        for i, y in enumerate(ys):
            outs[i].append(y)
    torch.cuda.synchronize()
    for i in range(len(lens)):
        got = torch.cat(outs[i], dim=1).cpu().double().numpy()
        assert np.array_equal(got, alone[i]), i


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_step_graph_replays_bitwise(prec):
    """Steps replaying the captured step graph equal one-by-one launches, step
    by step, with eager device work and synchronizations between replays; a
    step larger than the reserved workspace grows it and recaptures."""
    sc = _sc()
    m, w = weights_for("rave_b")
    g = sc.Model(m, w, prec)
    e = sc.Model(m, w, prec)
    g.reserve(24)
    g.enable_graph(6)
    rng = np.random.default_rng(9)
    steps = [[int(v) for v in rng.integers(1, 5, size=5)] for _ in range(5)]
    steps.insert(3, [8, 8, 8, 8, 8])            # 40 frames > 24 reserved: grows and recaptures
    xs = [scgen.stream_latents(16, sum(st[i] for st in steps), 60 + i) for i in range(5)]
    sg = [sc.Stream(g, 8) for _ in range(5)]
    se = [sc.Stream(e, 8) for _ in range(5)]
    pos = [0] * 5
    scratch = torch.zeros(1 << 20, device="cuda")
    for k, st in enumerate(steps):
        ins = [torch.from_numpy(np.ascontiguousarray(xs[i][:, pos[i]:pos[i] + st[i]])).cuda() for i in range(5)]
        for i in range(5):
            pos[i] += st[i]
        yg = sc.process_batch(g, sg, ins)
        scratch.mul_(0.5).add_(float(k))        # eager work between replays
        torch.cuda.synchronize()
        ye = sc.process_batch(e, se, ins)
        torch.cuda.synchronize()
        for i in range(5):
            assert torch.equal(yg[i], ye[i]), (k, i)
    log("step graph: %d steps bitwise equal (%s)" % (len(steps), prec))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_split_step_bitwise(prec):
    """A step of at least 32 streams and 512 input frames runs as two halves
    of its streams at once (the second half on an internal HIP stream, at a
    workspace offset); its outputs equal the same steps run as one launch
    sequence, step by step, including a step too small to split."""
    sc = _sc()
    m, w = weights_for("rave_b")
    scales = None
    if prec == "fp8":
        from paper_2204_07064_amd import calibrate
        scales = calibrate.act_scales(sc, m, w, [scgen.latents(16, 32, 1)])
    a = sc.Model(m, w, prec, act_scales=scales)
    b = sc.Model(m, w, prec, act_scales=scales, options=sc._native.SC_MODEL_NO_SPLIT)
    S = 64
    rng = np.random.default_rng(21)
    steps = [[int(v) for v in rng.choice([1, 2, 4, 8, 16, 32], size=S)] for _ in range(3)]
    steps.insert(1, [1] * S)                     # 64 frames: below the split threshold
    assert all(sum(st) >= 512 for k, st in enumerate(steps) if k != 1)
    xs = [scgen.stream_latents(16, sum(st[i] for st in steps), 300 + i) for i in range(S)]
    sa = [sc.Stream(a, 32) for _ in range(S)]
    sb = [sc.Stream(b, 32) for _ in range(S)]
    pos = [0] * S
    for k, st in enumerate(steps):
        ins = [torch.from_numpy(np.ascontiguousarray(xs[i][:, pos[i]:pos[i] + st[i]])).cuda() for i in range(S)]
        for i in range(S):
            pos[i] += st[i]
        ya = sc.process_batch(a, sa, ins)
        yb = sc.process_batch(b, sb, ins)
        torch.cuda.synchronize()
        for i in range(S):
            assert torch.equal(ya[i], yb[i]), (k, i)
    log("split steps: %d steps x %d streams bitwise equal (%s)" % (len(steps), S, prec))


@pytest.mark.parametrize("name,prec", [("rave_b", "fp32"), ("rave_b", "bf16"), ("rave_b", "fp8"),
                                       ("outconv", "fp32"), ("outconv", "bf16"),
                                       ("outconv64", "fp32"), ("outconv64", "bf16"),
                                       ("outconv48", "bf16")])   # (FP32 48-channel convs gather)
def test_output_conv_fusion_matches(name, prec):
    """The decoder's one-channel output conv computed in the epilogue of the
    last window conv (plus the tail launch for frames whose taps cross a tile
    boundary, and the move of its input cache) matches its own launch: streams
    that span several tiles, 1-frame buffers, warm-up masks, split and unsplit
    steps, state carried across steps.  Both add the same FP32 products of the
    same inputs, in different orders (the fused one by channel groups, the
    standalone one channel after channel), so they agree to FP32 rounding of
    a 224-term sum: 1e-5 absolute on outputs in (-1, 1), the FP32 bound
    against the oracle.  Masked frames are exact zeros in both."""
    sc = _sc()
    m, w = weights_for(name)
    C = m["in_channels"]
    scales = None
    if prec == "fp8":
        from paper_2204_07064_amd import calibrate
        scales = calibrate.act_scales(sc, m, w, [scgen.latents(C, 32, 1)])
    a = sc.Model(m, w, prec, act_scales=scales)
    b = sc.Model(m, w, prec, act_scales=scales, options=sc._native.SC_MODEL_NO_OUT_FUSION)
    S = 48
    rng = np.random.default_rng(33)
    steps = [[int(v) for v in rng.choice([1, 2, 3, 5, 8, 16, 32], size=S)] for _ in range(4)]
    steps.insert(1, [1] * S)                     # one tile per stream, below the split threshold
    xs = [scgen.stream_latents(C, sum(st[i] for st in steps), 700 + i) for i in range(S)]
    sa = [sc.Stream(a, 32, warmup_mask=(i % 3 == 0)) for i in range(S)]
    sb = [sc.Stream(b, 32, warmup_mask=(i % 3 == 0)) for i in range(S)]
    pos = [0] * S
    worst = 0.0
    for k, st in enumerate(steps):
        ins = [torch.from_numpy(np.ascontiguousarray(xs[i][:, pos[i]:pos[i] + st[i]])).cuda() for i in range(S)]
        for i in range(S):
            pos[i] += st[i]
        ya = sc.process_batch(a, sa, ins)
        yb = sc.process_batch(b, sb, ins)
        torch.cuda.synchronize()
        for i in range(S):
            assert torch.equal(ya[i] == 0, yb[i] == 0), (k, i)
            err = (ya[i] - yb[i]).abs().max().item()
            assert err <= 1e-5, (k, i, err)
            worst = max(worst, err)
    # the same streams as single-stream calls (one tile each, no tail frames),
    # timed per launch (which also runs steps unsplit)
    a.profile(True)
    for k in range(3):
        for i in range(0, S, 7):
            x = torch.from_numpy(np.ascontiguousarray(scgen.stream_latents(C, 1, 900 + 10 * k + i))).cuda()
            ya = sa[i].process(x)
            yb = sb[i].process(x)
            torch.cuda.synchronize()
            err = (ya - yb).abs().max().item()
            assert err <= 1e-5, (k, i, err)
            worst = max(worst, err)
    impls = [p["impl"] for p in a.profile_read()]
    assert impls[-1] == 3 and impls[-2] == 2, impls   # the fused pair ran
    a.profile(False)
    log("output conv fusion %s: %d steps x %d streams, max |fused - own launch| %.2e (%s)" % (
        name, len(steps), S, worst, prec))


@pytest.mark.parametrize("name,mult,prec", [("encoder", 128, "fp32"), ("encoder", 128, "bf16"),
                                            ("autoencoder", 128, "bf16"),
                                            ("branch3", 1, "fp32"), ("strided", 2, "fp32")])
def test_split_step_bitwise_other_models(name, mult, prec):
    """Split steps of the strided encoder (input frames a multiple of 128,
    workspace rates below one frame per input frame), of the four-branch unit
    (explicit delay lines) and of the strided unit equal one launch sequence."""
    sc = _sc()
    m, w = weights_for(name)
    a = sc.Model(m, w, prec)
    b = sc.Model(m, w, prec, options=sc._native.SC_MODEL_NO_SPLIT)
    C = m["in_channels"]
    S = 40
    rng = np.random.default_rng(33)
    choices = [mult * k for k in (4, 8, 16)] if mult > 1 else [8, 16, 24]
    steps = [[int(v) for v in rng.choice(choices, size=S)] for _ in range(3)]
    assert all(sum(st) >= 512 for st in steps)
    top = max(choices)
    xs = [scgen.stream_latents(C, sum(st[i] for st in steps), 700 + i) for i in range(S)]
    sa = [sc.Stream(a, top) for _ in range(S)]
    sb = [sc.Stream(b, top) for _ in range(S)]
    pos = [0] * S
    for k, st in enumerate(steps):
        ins = [torch.from_numpy(np.ascontiguousarray(xs[i][:, pos[i]:pos[i] + st[i]])).cuda() for i in range(S)]
        for i in range(S):
            pos[i] += st[i]
        ya = sc.process_batch(a, sa, ins)
        yb = sc.process_batch(b, sb, ins)
        torch.cuda.synchronize()
        for i in range(S):
            assert torch.equal(ya[i], yb[i]), (name, k, i)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_state_export_import_continues_bitwise(prec):
    """A stream checkpointed after some buffers and resumed in a fresh stream
    (of the same model object, or of a second model object: migration)
    continues bitwise as the uninterrupted stream."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    x = scgen.stream_latents(16, 24, 41)
    whole = run_stream(mod, x, [5, 7, 3, 9])
    a = sc.Stream(mod, 9)
    first = run_stream(mod, x[:, :12], [5, 7], stream=a)
    state = a.export_state()
    assert len(state) == sc.lib().sc_stream_state_bytes(mod.handle)
    for target in (mod, sc.Model(m, w, prec)):
        b = sc.Stream(target, 9)
        b.import_state(state)
        assert b.position == 12
        rest = run_stream(target, x[:, 12:], [3, 9], stream=b)
        assert np.array_equal(np.concatenate([first, rest], axis=1), whole)


def test_state_import_rejects_other_graph():
    sc = _sc()
    m, w = weights_for("rave_b")
    a = sc.Stream(sc.Model(m, w, "fp32"), 8)
    state = a.export_state()
    b = sc.Stream(sc.Model(m, w, "bf16"), 8)
    with pytest.raises(sc.ScError):
        b.import_state(state)                     # another precision
    with pytest.raises(sc.ScError):
        a.import_state(state[:-4])                # wrong size
    m3, w3 = weights_for("stack3")
    c = sc.Stream(sc.Model(m3, w3, "fp32"), 8)
    with pytest.raises(sc.ScError):
        c.import_state(state)                     # another graph


def test_bad_length_changes_nothing():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    st = sc.Stream(mod, 16)
    x = scgen.stream_latents(16, 32, 8)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty((1, 128 * 17), device="cuda")
    with pytest.raises(sc.ScError) as ei:
        st.process_into(xd[:, :17].contiguous(), out)       # above max_buffer_frames
    assert ei.value.status == -4
    with pytest.raises(sc.ScError):
        st.process_into(xd[:, :1].contiguous(), out, n_frames=0)
    assert st.position == 0
    a = run_stream(mod, x, [16, 16], stream=st)
    b = run_stream(mod, x, [16, 16])
    assert np.array_equal(a, b)


def test_encoder_rejects_misaligned_buffer():
    sc = _sc()
    m, w = weights_for("encoder")
    mod = sc.Model(m, w, "fp32")
    st = sc.Stream(mod, 256)
    x = torch.zeros((1, 100), device="cuda")
    with pytest.raises(sc.ScError) as ei:
        st.process(x)
    assert ei.value.status == -4
