"""GPU tests of failure paths and of paths checked against the FP64 oracle
beyond the plain stream: per-stream isolation (a NaN in one stream's input),
reset after it, the serving loop with buffers still queued at close and at
destroy, refused submissions and polls, FP8 scale handling around servers,
and the oracle on resumed (imported) streams and on served streams."""
import numpy as np
import pytest

import scgen
from gpu_helpers import log, oracle_compare, run_stream, weights_for
from oracle import metrics, offline

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
BF16_SNR = 40.0
SC_EINVAL, SC_ELENGTH, SC_ESTATE = -1, -4, -6


def _sc():
    import paper_2204_07064_amd as sc
    return sc


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batched_steps(sc, mod, streams, xs, lens):
    """lens[k][i]: frames of stream i at step k; xs: device tensors."""
    pos = [0] * len(xs)
    outs = [[] for _ in xs]
    for step in lens:
        ins = []
        for i, n in enumerate(step):
            ins.append(xs[i][:, pos[i]:pos[i] + n].contiguous())
            pos[i] += n
        for i, y in enumerate(sc.process_batch(mod, streams, ins)):
            outs[i].append(y)
    torch.cuda.synchronize()
    return [torch.cat(o, dim=1).cpu().double().numpy() for o in outs]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_nan_in_one_stream_is_isolated_and_reset_recovers(prec):
    """A NaN in one stream's input poisons only that stream: every other
    stream of the same batched steps is bitwise what it is without the NaN
    (each stream's cache is its own state), and stream_reset brings the
    poisoned stream back to exactly a fresh stream's output."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    S = 9
    rng = np.random.default_rng(12)
    lens = [[int(v) for v in rng.choice([1, 2, 5, 8, 16], size=S)] for _ in range(4)]
    frames = [sum(step[i] for step in lens) for i in range(S)]
    xs = [scgen.stream_latents(16, frames[i], 300 + i) for i in range(S)]
    bad = [x.copy() for x in xs]
    bad[4][3, 0] = np.nan                    # first frame of stream 4
    clean_out = _batched_steps(sc, mod, [sc.Stream(mod, 16) for _ in range(S)],
                               [torch.from_numpy(x).cuda() for x in xs], lens)
    streams = [sc.Stream(mod, 16) for _ in range(S)]
    dirty_out = _batched_steps(sc, mod, streams, [torch.from_numpy(x).cuda() for x in bad], lens)
    assert not np.all(np.isfinite(dirty_out[4]))
    for i in range(S):
        if i != 4:
            assert np.array_equal(dirty_out[i], clean_out[i]), i
    # the poisoned stream's caches hold NaN until reset
    streams[4].reset()
    assert streams[4].position == 0
    x4 = scgen.stream_latents(16, 24, 77)
    again = run_stream(mod, x4, [8, 16], stream=streams[4])
    fresh = run_stream(mod, x4, [8, 16])
    assert np.all(np.isfinite(again))
    assert np.array_equal(again, fresh)


def test_import_continuation_matches_oracle():
    """A stream exported after 3 buffers and resumed in a stream of another
    model object: the concatenated output (first part from the original,
    rest from the resumed stream) equals the FP64 offline model over the whole
    comparison window [c_L, T_out - D)."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    x = scgen.stream_latents(16, 40, 51)
    a = sc.Stream(mod, 16)
    first = run_stream(mod, x[:, :13], [4, 1, 8], stream=a)
    state = a.export_state()
    mod2 = sc.Model(m, w, "fp32")
    b = sc.Stream(mod2, 16)
    b.import_state(state)
    rest = run_stream(mod2, x[:, 13:], [16, 2, 9], stream=b)
    s = np.concatenate([first, rest], axis=1)
    err, snr, _ = oracle_compare(m, w, x, s, mod.latency, mod.warmup)
    log("resumed stream vs oracle: max-abs %.3e snr %.1f dB" % (err, snr))
    assert err <= FP32_TOL


def _serve_all(sc, mod, xs, lens, use_graph=True, max_buf=16):
    srv = sc.Server(mod, len(xs), max_buf, use_graph=use_graph)
    tickets = []
    for b in range(len(lens[0])):
        for i, x in enumerate(xs):
            a = sum(lens[i][:b])
            tickets.append((i, b, srv.submit(i, x[:, a:a + lens[i][b]])))
    srv.drain()
    outs = [[None] * len(lens[0]) for _ in xs]
    for i, b, t in tickets:
        outs[i][b] = srv.poll(t, lens[i][b])[0]
    srv.close()
    return [np.concatenate(o, axis=1).astype(np.float64) for o in outs]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_served_streams_match_oracle(prec):
    """Streams served in an interleaved mix (merged buffers, graph replays),
    compared with the FP64 offline model on sampled streams."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    rng = np.random.default_rng(19)
    S = 20
    lens = [[int(v) for v in rng.integers(1, 9, size=5)] for _ in range(S)]
    xs = [scgen.stream_latents(16, sum(l), 900 + i) for i, l in enumerate(lens)]
    outs = _serve_all(sc, mod, xs, lens)
    for i in (0, 7, 19):
        err, snr, _ = oracle_compare(m, w, xs[i], outs[i], mod.latency, mod.warmup)
        log("%s served stream %d (%d frames): max-abs %.3e snr %.1f dB" % (prec, i, sum(lens[i]), err, snr))
        if prec == "fp32":
            assert err <= FP32_TOL
        else:
            assert snr >= BF16_SNR


def test_server_close_and_destroy_with_buffers_queued():
    """Closing a stream that still has queued buffers lets them complete (and
    only then frees its slot, admitting a waiting stream); destroying a server
    with buffers still queued (admitted and waiting streams) returns, and the
    model keeps working afterwards."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    xs = [scgen.stream_latents(16, 24, 400 + i) for i in range(3)]
    srv = sc.Server(mod, 2, 8, use_graph=False)
    t = {}
    for i in range(3):                       # stream 2 waits for a slot
        for b in range(3):
            t[(i, b)] = srv.submit(i, xs[i][:, 8 * b:8 * b + 8])
    for i in range(3):
        srv.close_stream(i)                  # all three buffers of each still queued
    srv.drain()
    st = srv.stats()
    assert st["buffers"] == 9 and st["admitted"] == 0 and st["waiting"] == 0
    for i in range(3):
        got = np.concatenate([srv.poll(t[(i, b)], 8)[0] for b in range(3)], axis=1).astype(np.float64)
        assert np.array_equal(got, run_stream(mod, xs[i], [8, 8, 8])), i
    # a closed stream takes no more buffers; a new id opens a new stream
    srv.close()
    srv = sc.Server(mod, 1, 8, use_graph=True)
    for i in range(4):                       # one admitted, three waiting
        for b in range(3):
            srv.submit(i, xs[i % 3][:, 8 * b:8 * b + 8])
    srv.close()                              # destroy with buffers queued
    again = run_stream(mod, xs[0], [8, 16])
    assert np.array_equal(again, run_stream(mod, xs[0], [24]))


def test_server_refuses_bad_submissions_without_state_change():
    """A buffer that is not a whole number of the model's input granules, or
    longer than max_buffer_frames, or of the wrong channel count, is refused
    (SC_ELENGTH / ValueError) and queues nothing."""
    sc = _sc()
    m, w = weights_for("autoencoder")            # input multiple: 128 samples
    mod = sc.Model(m, w, "fp32")
    srv = sc.Server(mod, 4, 512, use_graph=False)
    x = scgen.stream_latents(1, 1024, 5)
    for n in (100, 129, 640):
        with pytest.raises(sc.ScError) as ei:
            srv.submit(0, x[:, :n])
        assert ei.value.status == SC_ELENGTH
    with pytest.raises(ValueError):
        srv.submit(0, np.zeros((2, 128), np.float32))
    st = srv.stats()
    assert st["queued"] == 0 and st["admitted"] == 0 and st["waiting"] == 0
    t = srv.submit(0, x[:, :256])
    srv.drain()
    # a poll buffer too small for the output is refused and keeps the ticket
    with pytest.raises(sc.ScError) as ei:
        srv.poll(t, 128)
    assert ei.value.status == SC_EINVAL
    got = srv.poll(t, 256)[0]
    assert np.array_equal(got.astype(np.float64), run_stream(mod, x[:, :256], [256]))
    srv.close()


def test_fp8_scales_and_servers():
    """A server refuses an FP8 model that has no activation scales; while a
    server that replays captured graphs uses a model, its scales cannot be
    replaced (the graphs hold them); after the server is gone they can."""
    sc = _sc()
    m, w = weights_for("rave_b")
    plan = scgen.fp8_plan(m)
    noscale = sc.Model(m, w, layer_precision=plan)
    with pytest.raises(sc.ScError) as ei:
        sc.Server(noscale, 4, 8)
    assert ei.value.status == SC_EINVAL
    scales = np.full(noscale.n_layers, 4.0, np.float32)
    mod = sc.Model(m, w, layer_precision=plan, act_scales=scales)
    srv = sc.Server(mod, 4, 8, use_graph=True)
    with pytest.raises(sc.ScError) as ei:
        mod.set_act_scales(scales * 2)
    assert ei.value.status == SC_ESTATE
    srv.close()
    mod.set_act_scales(scales * 2)


def test_oversize_step_is_refused():
    """A step whose per-launch item count would leave 32-bit indexing is
    refused with SC_ELENGTH before anything is enqueued."""
    sc = _sc()
    m, w = weights_for("wide")
    mod = sc.Model(m, w, "bf16")
    with pytest.raises(sc.ScError) as ei:
        mod.reserve(1024 * 86)               # 88k latent frames x 512 x 48 items
    assert ei.value.status == SC_ELENGTH
