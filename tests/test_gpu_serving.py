"""GPU tests of the serving loop: continuous batching with hipGraph replays,
admission by HBM budget, same-stream buffer merging, and each stream's result
equal (bitwise) to processing it alone."""
import numpy as np
import pytest

import scgen
from gpu_helpers import log, run_stream, weights_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sc():
    import paper_2204_07064_amd as sc
    return sc


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _workload(n_streams, n_bufs, seed, max_buf=8):
    rng = np.random.default_rng(seed)
    lens = [list(rng.integers(1, max_buf + 1, size=n_bufs)) for _ in range(n_streams)]
    xs = [scgen.stream_latents(16, int(sum(l)), 100 + i) for i, l in enumerate(lens)]
    # an arrival order that keeps each stream's buffers in order
    order = []
    nxt = [0] * n_streams
    while any(nxt[i] < n_bufs for i in range(n_streams)):
        i = int(rng.integers(0, n_streams))
        if nxt[i] < n_bufs:
            order.append((i, nxt[i]))
            nxt[i] += 1
    return lens, xs, order


def _serve(sc, mod, lens, xs, order, use_graph, budget=0, max_streams=None, close_after=True, max_buf=16):
    n = len(lens)
    srv = sc.Server(mod, max_streams or n, max_buf, hbm_budget_bytes=budget, use_graph=use_graph)
    tickets = {}
    starts = [np.concatenate([[0], np.cumsum(l)]) for l in lens]
    for (i, b) in order:
        a, e = int(starts[i][b]), int(starts[i][b + 1])
        tickets[(i, b)] = srv.submit(i, xs[i][:, a:e])
    if close_after:
        for i in range(n):
            srv.close_stream(i)
    srv.drain()
    outs = [[None] * len(l) for l in lens]
    lat = []
    for (i, b), t in tickets.items():
        r = srv.poll(t, int(lens[i][b]))
        assert r is not None
        outs[i][b] = r[0]
        lat.append(r[1])
    st = srv.stats()
    srv.close()
    return [np.concatenate(o, axis=1).astype(np.float64) for o in outs], lat, st


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_served_equals_alone(prec, use_graph):
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    lens, xs, order = _workload(24, 6, 1)
    outs, lat, st = _serve(sc, mod, lens, xs, order, use_graph)
    log("%s graph=%s: steps %d buffers %d merged %d, latency p50 %.2f ms"
        % (prec, use_graph, st["steps"], st["buffers"], st["merged_buffers"], 1e3 * np.median(lat)))
    assert st["buffers"] == 24 * 6
    assert min(lat) > 0
    for i in range(len(lens)):
        alone = run_stream(mod, xs[i], [int(v) for v in lens[i]])
        assert np.array_equal(outs[i], alone), i


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_served_split_steps_equal_alone(prec):
    """Steps of at least 32 streams and 512 frames run as two concurrent
    halves (launched one by one, next to the graph replays of small steps);
    every stream's output still equals its solo run."""
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, prec)
    rng = np.random.default_rng(17)
    S, B = 64, 4
    lens = [list(rng.integers(8, 17, size=B)) for _ in range(S)]
    xs = [scgen.stream_latents(16, int(sum(l)), 500 + i) for i, l in enumerate(lens)]
    order = [(i, b) for b in range(B) for i in range(S)]
    outs, lat, st = _serve(sc, mod, lens, xs, order, True, max_buf=32)
    log("%s split serving: steps %d buffers %d merged %d, %.0f frames per step"
        % (prec, st["steps"], st["buffers"], st["merged_buffers"], st["frames_in"] / max(st["steps"], 1)))
    assert st["buffers"] == S * B
    for i in range(S):
        alone = run_stream(mod, xs[i], [int(v) for v in lens[i]])
        assert np.array_equal(outs[i], alone), i


@pytest.mark.parametrize("use_graph", [True, False])
def test_served_audio_model_equals_alone(use_graph):
    """Audio in, audio out (the strided encoder feeding the decoder) through
    the server: buffers are whole 128-sample granules of the step's frame
    table, queued buffers merge, steps of 32+ streams split; every stream's
    output equals its solo run bit for bit."""
    sc = _sc()
    m, w = weights_for("autoencoder")
    mod = sc.Model(m, w, "bf16")
    rng = np.random.default_rng(23)
    S, B = 40, 3
    lens = [[128 * int(v) for v in rng.integers(1, 9, size=B)] for _ in range(S)]
    xs = [scgen.stream_latents(1, int(sum(l)), 800 + i) for i, l in enumerate(lens)]
    order = [(i, b) for b in range(B) for i in range(S)]
    outs, lat, st = _serve(sc, mod, lens, xs, order, use_graph, max_buf=128 * 16)
    log("audio model serving (graph %s): steps %d buffers %d merged %d"
        % (use_graph, st["steps"], st["buffers"], st["merged_buffers"]))
    assert st["buffers"] == S * B
    for i in range(S):
        alone = run_stream(mod, xs[i], lens[i])
        assert np.array_equal(outs[i], alone), i


def test_graph_replays_equal_eager():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "bf16")
    lens, xs, order = _workload(12, 10, 2)
    a, _, _ = _serve(sc, mod, lens, xs, order, True)
    b, _, _ = _serve(sc, mod, lens, xs, order, False)
    for i in range(len(lens)):
        assert np.array_equal(a[i], b[i])


def test_budget_admission_fifo():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "bf16")
    probe = sc.Server(mod, 8, 16)
    st0 = probe.stats()
    probe.close()
    budget = st0["fixed_bytes"] + int(3.5 * st0["per_stream_bytes"])
    srv = sc.Server(mod, 8, 16, hbm_budget_bytes=budget)
    assert srv.stats()["max_admitted"] == 3
    lens, xs, _ = _workload(8, 3, 3)
    starts = [np.concatenate([[0], np.cumsum(l)]) for l in lens]
    tickets = {}
    for i in range(8):                      # streams arrive in id order: FIFO admission
        for b in range(3):
            tickets[(i, b)] = srv.submit(i, xs[i][:, int(starts[i][b]):int(starts[i][b + 1])])
    done_order = []
    for i in range(8):
        srv.close_stream(i)
    srv.drain()
    st = srv.stats()
    assert st["buffers"] == 24 and st["admitted"] == 0 and st["waiting"] == 0
    for i in range(8):
        got = np.concatenate([srv.poll(tickets[(i, b)], int(lens[i][b]))[0] for b in range(3)], axis=1)
        alone = run_stream(mod, xs[i], [int(v) for v in lens[i]])
        assert np.array_equal(got.astype(np.float64), alone)
        done_order.append(i)
    srv.close()


def test_budget_too_small_is_refused():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "bf16")
    with pytest.raises(sc.ScError) as ei:
        sc.Server(mod, 8, 16, hbm_budget_bytes=1024)
    assert ei.value.status == -3


def test_submit_batch_and_latency_log():
    sc = _sc()
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "bf16")
    lens, xs, order = _workload(16, 5, 4)
    starts = [np.concatenate([[0], np.cumsum(l)]) for l in lens]
    bufs = []
    for (i, b) in order:
        bufs.append(np.ascontiguousarray(xs[i][:, int(starts[i][b]):int(starts[i][b + 1])], dtype=np.float32))
    ids = np.array([i for i, _ in order], np.int64)
    ptrs = np.array([x.ctypes.data for x in bufs], np.uint64)
    fr = np.array([x.shape[1] for x in bufs], np.int32)
    srv = sc.Server(mod, 16, 16)
    half = len(order) // 2
    t_keep = srv.submit_batch(ids[:half], ptrs[:half], fr[:half], discard=False)
    t_disc = srv.submit_batch(ids[half:], ptrs[half:], fr[half:], discard=True)
    srv.drain()
    tick, lat = srv.latencies()
    assert sorted(tick.tolist()) == sorted(t_disc.tolist())
    assert np.all(lat > 0)
    got = {}
    for k in range(half):
        got[order[k]] = srv.poll(int(t_keep[k]), int(fr[k]))[0]
    srv.close()
    # the kept outputs equal the first buffers of each stream processed alone
    for i in range(16):
        mine = [b for (j, b) in order[:half] if j == i]
        if not mine:
            continue
        alone = run_stream(mod, xs[i], [int(v) for v in lens[i]])
        n_out = sum(int(lens[i][b]) for b in mine) * 128
        ref = alone[:, :n_out]
        assert np.array_equal(np.concatenate([got[(i, b)] for b in mine], axis=1).astype(np.float64), ref)
