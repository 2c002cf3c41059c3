"""Streaming non-causal convolutions on MI355X (gfx950).

Python binding of the HIP library ``libstreamconv.so`` (C ABI in
``include/streamconv.h``).  The binding only marshals arguments: PyTorch
supplies device memory and HIP streams, every step of the computation runs in
the library's kernels.

    model = Model(node_list_model, weights_f32, precision="bf16")
    s = Stream(model, max_buffer_frames=32)
    y = s.process(x)          # x: cuda float32 [in_channels][T]
"""
import atexit
import ctypes

import numpy as np

from . import _native
from ._native import ScError, check, lib, nodes_array  # noqa: F401

__all__ = ["Model", "Stream", "Server", "BatchCall", "process_batch", "offline_batch", "ola_process", "plan",
           "ScError", "lib"]


_EXITING = [False]


@atexit.register
def _at_exit():
    # objects still alive at interpreter exit are left to the process teardown:
    # the HIP runtime may already be gone when their finalizers would run
    _EXITING[0] = True


def _stream_handle(hip_stream):
    if hip_stream is not None:
        return ctypes.c_void_p(int(hip_stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_device_buffer(t, channels, what, frames=None):
    """A device tensor the library reads or writes through a raw pointer:
    CUDA (HIP) float32, contiguous, [channels][>= frames]."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % what)
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("%s must be contiguous float32" % what)
    if t.dim() != 2 or t.shape[0] != channels:
        raise ValueError("%s must be [%d][frames], got %s" % (what, channels, tuple(t.shape)))
    if frames is not None and t.shape[1] < frames:
        raise ValueError("%s must hold at least %d frames, got %d" % (what, frames, t.shape[1]))


def plan(model):
    """Host-only planning (no GPU): latency, warm-up window, state bytes..."""
    arr = nodes_array(model)
    info = _native.ScModelInfo()
    check(lib().sc_plan(arr, len(arr), ctypes.byref(info)))
    return _native.info_dict(info)


class Model:
    def __init__(self, model, weights, precision="fp32", act_scales=None, options=0, device=0,
                 layer_precision=None):
        """layer_precision: optional list of "fp32" / "bf16" / "fp8", one per
        conv / transposed conv in node order (sc_model_create_mixed); then
        `precision` is ignored and reported as the lowest one used."""
        L = lib()
        self.spec = model
        arr = nodes_array(model)
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
        self._w = w
        sc = None
        if act_scales is not None:
            sc = np.ascontiguousarray(np.asarray(act_scales, dtype=np.float32))
        scp = sc.ctypes.data_as(_native.c_fp) if sc is not None else None
        h = ctypes.c_void_p()
        if layer_precision is None:
            check(L.sc_model_create(arr, len(arr), w.ctypes.data_as(_native.c_fp), w.size,
                                    _native.PRECISION[precision], scp, int(options), int(device),
                                    ctypes.byref(h)))
        else:
            lp = (ctypes.c_int32 * max(len(layer_precision), 1))(*[_native.PRECISION[p] for p in layer_precision])
            check(L.sc_model_create_mixed(arr, len(arr), w.ctypes.data_as(_native.c_fp), w.size, lp, scp,
                                          int(options), int(device), ctypes.byref(h)))
            precision = max(layer_precision, key=lambda p: _native.PRECISION[p]) if layer_precision else "fp32"
        self.handle = h
        self.layer_precision = None if layer_precision is None else list(layer_precision)
        self.precision = precision
        self.device = device
        info = _native.ScModelInfo()
        check(L.sc_model_info_get(h, ctypes.byref(info)))
        self.info = _native.info_dict(info)
        self.n_layers = L.sc_model_n_layers(h)

    @property
    def latency(self):
        return self.info["latency"]

    @property
    def warmup(self):
        return self.info["warmup"]

    def out_frames(self, n_frames):
        return n_frames * self.info["out_num"] // self.info["out_den"]

    def set_act_scales(self, scales):
        sc = np.ascontiguousarray(np.asarray(scales, dtype=np.float32))
        assert sc.size == self.n_layers
        check(lib().sc_model_set_act_scales(self.handle, sc.ctypes.data_as(_native.c_fp)))

    def enable_amax(self, on=True):
        check(lib().sc_model_enable_amax(self.handle, int(bool(on))))

    def read_amax(self, reset=False):
        out = np.zeros(max(self.n_layers, 1), np.float32)
        check(lib().sc_model_read_amax(self.handle, out.ctypes.data_as(_native.c_fp), int(bool(reset))))
        return out[:self.n_layers]

    def calibrated_scales(self):
        """Static FP8 activation scales from the maxima recorded so far
        (sc_model_calibrated_scales)."""
        out = np.zeros(max(self.n_layers, 1), np.float32)
        check(lib().sc_model_calibrated_scales(self.handle, out.ctypes.data_as(_native.c_fp)))
        return out[:self.n_layers]

    def profile(self, enable=True):
        check(lib().sc_model_profile(self.handle, int(bool(enable))))

    def profile_read(self):
        n = ctypes.c_int32()
        check(lib().sc_model_profile_read(self.handle, None, 0, ctypes.byref(n)))
        arr = (_native.ScOpProfile * max(n.value, 1))()
        check(lib().sc_model_profile_read(self.handle, arr, n.value, ctypes.byref(n)))
        return [{f: getattr(arr[i], f) for f, _ in _native.ScOpProfile._fields_} for i in range(n.value)]

    def enable_graph(self, max_streams):
        """Replay one captured graph per step of up to max_streams streams (0: off)."""
        check(lib().sc_model_enable_graph(self.handle, int(max_streams)))

    def reserve(self, max_step_frames):
        """Size the workspace for steps of up to max_step_frames input frames."""
        check(lib().sc_model_reserve(self.handle, int(max_step_frames)))

    def close(self):
        if self.handle and not _EXITING[0]:
            lib().sc_model_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    def __init__(self, model, max_buffer_frames, warmup_mask=False, hip_stream=None):
        self.model = model
        self.max_buffer_frames = int(max_buffer_frames)
        h = ctypes.c_void_p()
        flags = _native.SC_FLAG_WARMUP_MASK if warmup_mask else 0
        check(lib().stream_create(model.handle, self.max_buffer_frames, flags,
                                  _stream_handle(hip_stream), ctypes.byref(h)))
        self.handle = h

    def process_into(self, x, out, n_frames=None, hip_stream=None):
        """x: cuda float32 [C_in][T]; out: cuda float32 [C_out][T_out]."""
        T = int(x.shape[-1]) if n_frames is None else int(n_frames)
        info = self.model.info
        _check_device_buffer(x, info["in_channels"], "input", T)
        _check_device_buffer(out, info["out_channels"], "output", self.model.out_frames(T))
        check(lib().stream_process(self.handle, ctypes.c_void_p(x.data_ptr()), T,
                                   ctypes.c_void_p(out.data_ptr()), _stream_handle(hip_stream)))
        return out

    def process_into_noalloc(self, x, out, n_frames=None, hip_stream=None):
        """process_into through stream_process_noalloc: the step's workspace
        in the library's fixed scratch array (no device allocation)."""
        T = int(x.shape[-1]) if n_frames is None else int(n_frames)
        info = self.model.info
        _check_device_buffer(x, info["in_channels"], "input", T)
        _check_device_buffer(out, info["out_channels"], "output", self.model.out_frames(T))
        check(lib().stream_process_noalloc(self.handle, ctypes.c_void_p(x.data_ptr()), T,
                                           ctypes.c_void_p(out.data_ptr()), _stream_handle(hip_stream)))
        return out

    def process(self, x, hip_stream=None):
        import torch
        _check_device_buffer(x, self.model.info["in_channels"], "input")
        T = int(x.shape[-1])
        out = torch.empty((self.model.info["out_channels"], self.model.out_frames(T)),
                          dtype=torch.float32, device=x.device)
        return self.process_into(x, out, T, hip_stream)

    def reset(self, hip_stream=None):
        check(lib().stream_reset(self.handle, _stream_handle(hip_stream)))

    @property
    def position(self):
        return lib().stream_position(self.handle)

    def export_state(self):
        """The stream's whole state as bytes (after its queued steps)."""
        n = lib().sc_stream_state_bytes(self.model.handle)
        buf = ctypes.create_string_buffer(n)
        check(lib().stream_export(self.handle, buf, n))
        return buf.raw

    def import_state(self, state):
        """Continue from an exported state (same graph and precision)."""
        b = bytes(state)
        check(lib().stream_import(self.handle, ctypes.c_char_p(b), len(b)))

    def close(self):
        if self.handle and not _EXITING[0]:
            lib().stream_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def process_batch(model, streams, xs, outs=None, hip_stream=None):
    """One batched step: buffer xs[i] (cuda [C_in][T_i]) for streams[i]."""
    import torch
    n = len(streams)
    if len(xs) != n or (outs is not None and len(outs) != n):
        raise ValueError("streams, inputs and outputs differ in length")
    for x in xs:
        _check_device_buffer(x, model.info["in_channels"], "input")
    if outs is None:
        outs = [torch.empty((model.info["out_channels"], model.out_frames(int(x.shape[-1]))),
                            dtype=torch.float32, device=x.device) for x in xs]
    for x, o in zip(xs, outs):
        _check_device_buffer(o, model.info["out_channels"], "output", model.out_frames(int(x.shape[-1])))
    sh = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
    ins = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    ous = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    tf = (ctypes.c_int32 * n)(*[int(x.shape[-1]) for x in xs])
    check(lib().sc_process_batch(model.handle, n, sh, ins, tf, ous, _stream_handle(hip_stream)))
    return outs


def offline_batch(model, xs, outs=None, hip_stream=None):
    """The model offline (zero-padded at both ends, no latency) on each
    buffer xs[i] (cuda [C_in][T_i]): outputs cuda [C_out][T_i * out_rate]."""
    import torch
    n = len(xs)
    if n == 0 or (outs is not None and len(outs) != n):
        raise ValueError("no buffers, or inputs and outputs differ in length")
    for x in xs:
        _check_device_buffer(x, model.info["in_channels"], "input")
    if outs is None:
        outs = [torch.empty((model.info["out_channels"], model.out_frames(int(x.shape[-1]))),
                            dtype=torch.float32, device=x.device) for x in xs]
    for x, o in zip(xs, outs):
        _check_device_buffer(o, model.info["out_channels"], "output", model.out_frames(int(x.shape[-1])))
    ins = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    ous = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    tf = (ctypes.c_int32 * n)(*[int(x.shape[-1]) for x in xs])
    check(lib().sc_offline_batch(model.handle, n, ins, tf, ous, _stream_handle(hip_stream)))
    return outs


def ola_process(model, x, window, overlap, out=None, hip_stream=None):
    """The overlap-add baseline over the whole signal x (cuda [C_in][T]):
    buffers of `window` input frames every window - overlap frames, each
    evaluated offline, tapered and summed; output cuda [C_out][T * out_rate]."""
    import torch
    _check_device_buffer(x, model.info["in_channels"], "input")
    T = int(x.shape[-1])
    if out is None:
        out = torch.empty((model.info["out_channels"], model.out_frames(T)), dtype=torch.float32, device=x.device)
    _check_device_buffer(out, model.info["out_channels"], "output", model.out_frames(T))
    check(lib().sc_ola_process(model.handle, ctypes.c_void_p(x.data_ptr()), T, int(window), int(overlap),
                               ctypes.c_void_p(out.data_ptr()), _stream_handle(hip_stream)))
    return out


class BatchCall:
    """Prebuilt arguments of one batched step (streams, device input and
    output addresses, frames), so that issuing the step costs one library
    call.  The buffers behind the addresses must stay alive."""

    def __init__(self, model, streams, in_ptrs, frames, out_ptrs):
        n = len(streams)
        if not (len(in_ptrs) == len(frames) == len(out_ptrs) == n):
            raise ValueError("streams, inputs, frames and outputs differ in length")
        self.model = model
        self.n = n
        self.sh = (ctypes.c_void_p * n)(*[s.handle.value for s in streams])
        self.ins = (ctypes.c_void_p * n)(*[int(p) for p in in_ptrs])
        self.tf = (ctypes.c_int32 * n)(*[int(f) for f in frames])
        self.ous = (ctypes.c_void_p * n)(*[int(p) for p in out_ptrs])

    def run(self, hip_stream=None):
        check(lib().sc_process_batch(self.model.handle, self.n, self.sh, self.ins, self.tf, self.ous,
                                     _stream_handle(hip_stream)))


class Server:
    """Continuous-batching server over one model (see sc_server_* in the
    header).  Inputs and outputs are host numpy arrays; the server copies them."""

    def __init__(self, model, max_streams, max_buffer_frames, hbm_budget_bytes=0, use_graph=True,
                 warmup_mask=False):
        cfg = _native.ScServerConfig(int(max_streams), int(max_buffer_frames), int(hbm_budget_bytes),
                                     int(bool(use_graph)),
                                     _native.SC_FLAG_WARMUP_MASK if warmup_mask else 0)
        h = ctypes.c_void_p()
        check(lib().sc_server_create(model.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.model = model
        self.cin = model.info["in_channels"]
        self.cout = model.info["out_channels"]

    def submit(self, stream_id, x):
        """x: float32 [in_channels][frames] (host).  Returns a ticket."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        if x.ndim != 2 or x.shape[0] != self.cin:
            raise ValueError("input must be [%d][frames], got %s" % (self.cin, x.shape))
        t = ctypes.c_int64()
        check(lib().sc_server_submit(self.handle, int(stream_id), x.ctypes.data_as(_native.c_fp), x.shape[-1],
                                     ctypes.byref(t)))
        return t.value

    def submit_batch(self, stream_ids, ptrs, frames, discard=True):
        """Queue len(stream_ids) buffers under one lock.  ptrs: host addresses
        (int64/uint64 numpy array) of float32 [in_channels][frames[i]] buffers
        that stay alive for the call.  Returns the tickets; with discard no
        output is kept and (ticket, latency) goes to latencies()."""
        ids = np.ascontiguousarray(stream_ids, dtype=np.int64)
        p = np.ascontiguousarray(ptrs, dtype=np.uint64)
        f = np.ascontiguousarray(frames, dtype=np.int32)
        n = len(ids)
        if len(p) != n or len(f) != n:
            raise ValueError("stream_ids, ptrs and frames differ in length")
        t = np.empty(n, np.int64)
        check(lib().sc_server_submit_batch(
            self.handle, n, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            p.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p)), f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            _native.SC_SUBMIT_DISCARD if discard else 0,
            t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return t

    def latencies(self, max_n=1 << 20):
        """(tickets, latency_s) of finished discarded buffers, completion order."""
        t = np.empty(max_n, np.int64)
        lat = np.empty(max_n, np.float64)
        n = ctypes.c_int64()
        check(lib().sc_server_latencies(self.handle, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), max_n,
                                        ctypes.byref(n)))
        return t[:n.value], lat[:n.value]

    def poll(self, ticket, frames):
        """(output [out_channels][frames*rate], latency_s) when done, else None
        (the library refuses a `frames` smaller than the buffer's)."""
        out = np.empty((self.cout, self.model.out_frames(frames)), np.float32)
        lat = ctypes.c_double()
        st = lib().sc_server_poll(self.handle, int(ticket), out.ctypes.data_as(_native.c_fp), out.size,
                                  ctypes.byref(lat))
        if st == _native.SC_PENDING:
            return None
        check(st)
        return out, lat.value

    def close_stream(self, stream_id):
        check(lib().sc_server_close_stream(self.handle, int(stream_id)))

    def drain(self):
        check(lib().sc_server_drain(self.handle))

    def stats(self):
        st = _native.ScServerStats()
        check(lib().sc_server_stats_get(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _native.ScServerStats._fields_}

    def close(self):
        if self.handle and not _EXITING[0]:
            lib().sc_server_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
