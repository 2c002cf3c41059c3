"""The bench's algorithmic FLOP and byte accounting (host logic, no GPU):
a window conv that computes the layer before it in its own launch (a
transposed conv, or the first conv of a fused residual pair) is charged both
layers' FLOPs, the first layer's input, state and weights, and not the first
layer's output, which never reaches memory."""
import bench


def _ops():
    ct = {"node": 23, "kind": 2, "impl": 1, "precision": 1, "cin": 64, "cout": 32, "k": 4, "stride": 2,
          "cache_len": 2, "dilation": 1, "launches": 0, "frames_in": 0, "frames_out": 0, "entries": 0, "ms": 0.0}
    cv = {"node": 25, "kind": 1, "impl": 2, "precision": 1, "cin": 32, "cout": 32, "k": 3, "stride": 1,
          "cache_len": 2, "dilation": 1, "launches": 10, "frames_in": 344064 * 10, "frames_out": 344064 * 10,
          "entries": 2560, "ms": 0.38}
    return ct, cv


def test_fused_producer_is_found_only_without_launches():
    ct, cv = _ops()
    assert bench.fused_producer([ct, cv], cv) is ct
    assert bench.fused_tail([ct, cv], cv) is None
    ct2 = dict(ct, launches=10)
    assert bench.fused_producer([ct2, cv], cv) is None


def test_fused_pair_accounting():
    ct, cv = _ops()
    f_cv, b_cv = bench.op_accounting(cv)
    x = cv["frames_in"]
    # the transposed conv as its own layer over the same frames
    alone = dict(ct, frames_in=x // 2, frames_out=x, entries=cv["entries"], launches=cv["launches"])
    f_ct, b_ct = bench.op_accounting(alone)
    f, b = bench.op_accounting(cv, ct=ct)
    # FLOPs: 2 MACs per output element and tap: conv 3 taps x 32 in, convT 2 taps x 64 in
    assert f_cv == 2.0 * x * 32 * 32 * 3
    assert f_ct == 2.0 * x * 32 * 2 * 64
    assert f == f_cv + f_ct
    # bytes: both layers less the transposed conv's output written and read back (FP32)
    assert b == b_cv + b_ct - 2 * 4.0 * x * 32
    assert b < b_cv + b_ct


def test_roofline_names_the_pair():
    ct, cv = _ops()
    r = bench.roofline([ct, cv])
    assert r["bound"] == "hbm" and "transposed conv node 23" in r["kernel"]
    assert r["flops_per_launch"] == round(bench.op_accounting(cv, ct=ct)[0] / cv["launches"])


def _pair():
    a = {"node": 18, "kind": 1, "impl": 2, "precision": 1, "cin": 64, "cout": 64, "k": 3, "stride": 1,
         "cache_len": 2, "dilation": 1, "launches": 0, "frames_in": 0, "frames_out": 0, "entries": 0, "ms": 0.0}
    b = {"node": 20, "kind": 1, "impl": 2, "precision": 1, "cin": 64, "cout": 64, "k": 3, "stride": 1,
         "cache_len": 6, "dilation": 3, "launches": 10, "frames_in": 172032 * 10, "frames_out": 172032 * 10,
         "entries": 2560, "ms": 0.47}
    return a, b


def test_residual_pair_accounting():
    a, b = _pair()
    assert bench.fused_producer([a, b], b) is a
    x = b["frames_in"]
    f_b, b_b = bench.op_accounting(b)
    f_a, b_a = bench.op_accounting(dict(a, frames_in=x, frames_out=x, entries=b["entries"], launches=b["launches"]))
    f, byts = bench.op_accounting(b, ct=a)
    assert f_a == f_b == 2.0 * x * 64 * 64 * 3
    assert f == f_a + f_b
    # the first conv's output (FP32) is neither written nor read back
    assert byts == b_a + b_b - 2 * 4.0 * x * 64
    r = bench.roofline([a, b])
    assert "residual conv node 18" in r["kernel"]
    assert r["bound"] == "mfma" and r["flops_per_launch"] == round(f / b["launches"])


def test_measured_traffic_only_for_its_model():
    """The counter table holds the headline decoder's nodes: another model's
    node of the same number and kernel family gets no traffic figure."""
    n, rec = next(iter(bench.MEASURED_TRAFFIC["by_node"].items()))
    impl = {v: k for k, v in bench.IMPL_NAME.items()}[rec[0]]
    best = {"node": n, "impl": impl, "precision": 1}
    assert bench.measured_traffic(best, "wide") is None
    assert bench.measured_traffic(best, "autoencoder") is None


def test_pair_with_fused_output_conv_accounting():
    """A pair whose second conv also computes the one-channel output conv:
    neither conv's 32-channel output reaches HBM, only the model output."""
    a, b = _pair()
    a = dict(a, cin=32, cout=32, node=27, dilation=3, cache_len=6)
    b = dict(b, cin=32, cout=32, node=29, dilation=9, cache_len=18, frames_in=344064 * 10,
             frames_out=344064 * 10)
    t = {"node": 30, "kind": 1, "impl": 3, "precision": 0, "cin": 32, "cout": 1, "k": 7, "stride": 1,
         "cache_len": 6, "dilation": 1, "launches": 10, "frames_in": 344064 * 10, "frames_out": 344064 * 10,
         "entries": 2560, "ms": 0.06}
    prof = [a, b, t]
    assert bench.fused_tail(prof, b) is t and bench.fused_producer(prof, b) is a
    x = b["frames_in"]
    f, byts = bench.op_accounting(b, tail=t, ct=a)
    f_b, b_b = bench.op_accounting(b, tail=t)
    f_a, b_a = bench.op_accounting(dict(a, frames_in=x, frames_out=x, entries=b["entries"], launches=b["launches"]))
    assert f == f_a + f_b == 2.0 * x * 32 * (32 * 3 * 2 + 7)
    assert byts == b_a + b_b - 2 * 4.0 * x * 32
    # the input of the first conv, the model output, caches and weights: no 32-channel output
    assert byts < 4.0 * x * 32 + 4.0 * x * 1 + 4.0 * b["entries"] * 32 * 64 + 10 * 1e5
    r = bench.roofline(prof)
    assert "output conv node 30" in r["kernel"] and r["bound"] == "hbm"
    assert r["layer_bytes_per_launch"] == round(byts / 10)
