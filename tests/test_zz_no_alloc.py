"""stream_process_noalloc (the entry point for callers that cannot allocate):
the same output as stream_process on the same stream history, bitwise, over
calls of decreasing size, and the oracle's result within the FP32 bound; a
buffer whose workspace does not fit the fixed scratch array is refused
with no state change."""
import numpy as np
import pytest

import scgen
from gpu_helpers import log, oracle_compare, weights_for

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair_run(mod, x, splits):
    """The same buffers through stream_process (stream a) and
    stream_process_noalloc (stream b); both outputs as float64 numpy."""
    import paper_2204_07064_amd as sc
    cap = max(splits)
    a = sc.Stream(mod, cap)
    b = sc.Stream(mod, cap)
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    oa, ob = [], []
    pos = 0
    for n in splits:
        xi = xd[:, pos:pos + n].contiguous()
        out_a = torch.empty((mod.info["out_channels"], mod.out_frames(n)), device="cuda")
        # poison the output so that a sample the call fails to write shows
        out_b = torch.full((mod.info["out_channels"], mod.out_frames(n)), float("nan"), device="cuda")
        a.process_into(xi, out_a)
        b.process_into_noalloc(xi, out_b)
        oa.append(out_a)
        ob.append(out_b)
        pos += n
    torch.cuda.synchronize()
    assert a.position == b.position == pos
    res = (torch.cat(oa, dim=1).cpu().double().numpy(), torch.cat(ob, dim=1).cpu().double().numpy())
    a.close()
    b.close()
    return res


@pytest.mark.parametrize("name,prec,splits", [
    ("rave_b", "fp32", [24, 5]),          # two calls, the second smaller
    ("rave_b", "bf16", [32, 7, 1]),
    ("autoencoder", "fp32", [128 * 16, 128 * 8]),
    ("stack3", "fp32", [4096, 512]),
])
def test_noalloc_equals_stream_process(name, prec, splits):
    import paper_2204_07064_amd as sc
    log("noalloc %s %s splits=%s" % (name, prec, splits))
    m, w = weights_for(name)
    x = scgen.stream_latents(m["in_channels"], sum(splits), 0)
    mod = sc.Model(m, w, prec)
    sa, sb = _pair_run(mod, x, splits)
    assert np.isfinite(sb).all()
    assert np.array_equal(sa, sb)
    if prec == "fp32":
        err, snr, _ = oracle_compare(m, w, x, sb, mod.latency, mod.warmup)
        log("  max-abs %.3e snr %.1f dB" % (err, snr))
        assert err <= FP32_TOL


def test_noalloc_oversize_is_refused_without_state_change():
    import paper_2204_07064_amd as sc
    from paper_2204_07064_amd import _native as n
    m, w = weights_for("rave_b")
    mod = sc.Model(m, w, "fp32")
    big = 4096       # stage-4 activations alone: 4096 x 128 frames x 32 ch x 4 B = 64 MiB
    st = sc.Stream(mod, big)
    x = torch.zeros((m["in_channels"], big), device="cuda")
    out = torch.empty((1, mod.out_frames(big)), device="cuda")
    with pytest.raises(sc.ScError) as ei:
        st.process_into_noalloc(x, out)
    assert n.STATUS[ei.value.status] == "SC_ELENGTH"
    assert st.position == 0
    # the stream still works, on both entry points
    y = scgen.stream_latents(m["in_channels"], 8, 0)
    yd = torch.from_numpy(y).cuda()
    o1 = torch.empty((1, mod.out_frames(8)), device="cuda")
    st.process_into_noalloc(yd, o1)
    o2 = st.process(yd)
    torch.cuda.synchronize()
    assert st.position == 16 and torch.isfinite(o1).all() and torch.isfinite(o2).all()
    st.close()
