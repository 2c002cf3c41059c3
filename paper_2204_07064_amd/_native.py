"""ctypes binding of ``libstreamconv.so`` (argument marshalling only).

Every function of ``include/streamconv.h`` is exposed under the same name on
the object returned by :func:`lib`.  Loading fails loudly when the library
has not been built: there is no fallback implementation.
"""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libstreamconv.so")

c_i32 = ctypes.c_int32
c_u32 = ctypes.c_uint32
c_i64 = ctypes.c_int64
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p
c_fp = ctypes.POINTER(ctypes.c_float)

SC_OK = 0
STATUS = {0: "SC_OK", -1: "SC_EINVAL", -2: "SC_ENOMEM", -3: "SC_EBUDGET", -4: "SC_ELENGTH",
          -5: "SC_EDEVICE", -6: "SC_ESTATE", -7: "SC_EUNSUPPORTED"}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2}
SC_FLAG_WARMUP_MASK = 1
SC_MODEL_NO_FUSION = 1
SC_MODEL_NO_MFMA = 2
SC_MODEL_NO_TWIN = 4
SC_MODEL_NO_WIN = 8
SC_MODEL_NO_SPLIT = 16
SC_MODEL_NO_OUT_FUSION = 32
SC_MODEL_NO_CONVT_FUSION = 64
SC_MODEL_NO_INPUT_DIRECT = 128
SC_MODEL_NO_PAIR_FUSION = 256
OPS = {"input": 0, "conv": 1, "convt": 2, "add": 3}

# every symbol the header declares (checked by the CPU test suite)
EXPORTS = [
    "sc_plan", "sc_model_create", "sc_model_info_get", "sc_model_n_layers",
    "sc_model_set_act_scales", "sc_model_read_amax", "sc_model_enable_amax", "sc_model_destroy",
    "stream_create", "stream_process", "stream_reset", "stream_position", "stream_destroy",
    "sc_process_batch", "sc_last_error", "sc_model_profile", "sc_model_profile_read",
    "sc_server_create", "sc_server_submit", "sc_server_poll", "sc_server_close_stream", "sc_server_drain",
    "sc_server_stats_get", "sc_server_destroy", "sc_server_submit_batch", "sc_server_latencies",
    "sc_model_reserve", "sc_model_enable_graph", "sc_stream_state_bytes", "stream_export", "stream_import",
    "sc_model_create_mixed", "sc_model_calibrated_scales", "stream_process_noalloc",
    "sc_offline_batch", "sc_ola_process",
]
SC_PENDING = 1
SC_SUBMIT_DISCARD = 1
SC_NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024


class ScNode(ctypes.Structure):
    _fields_ = [("op", c_i32), ("src", c_i32), ("src2", c_i32), ("cin", c_i32), ("cout", c_i32),
                ("k", c_i32), ("dilation", c_i32), ("stride", c_i32), ("pad_l", c_i32),
                ("pad_r", c_i32), ("pre_act", c_i32), ("post_act", c_i32)]


class ScModelInfo(ctypes.Structure):
    _fields_ = [("in_channels", c_i32), ("out_channels", c_i32), ("out_num", c_i32),
                ("out_den", c_i32), ("input_multiple", c_i32), ("n_launch", c_i32),
                ("latency", c_i64), ("warmup", c_i64), ("state_bytes_per_stream", c_i64),
                ("state_alloc_per_stream", c_i64), ("weight_bytes", c_i64)]


class ScOpProfile(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("impl", c_i32), ("precision", c_i32), ("node", c_i32),
                ("cin", c_i32), ("cout", c_i32), ("k", c_i32), ("dilation", c_i32), ("stride", c_i32),
                ("cache_len", c_i32), ("residual", c_i32), ("a0", c_i32), ("a1", c_i32),
                ("rate_in_num", c_i32), ("rate_in_den", c_i32), ("rate_out_num", c_i32),
                ("rate_out_den", c_i32), ("ms", ctypes.c_double), ("launches", c_i64),
                ("frames_in", c_i64), ("frames_out", c_i64), ("entries", c_i64)]


class ScServerConfig(ctypes.Structure):
    _fields_ = [("max_streams", c_i32), ("max_buffer_frames", c_i32), ("hbm_budget_bytes", c_i64),
                ("use_graph", c_i32), ("stream_flags", c_u32)]


class ScServerStats(ctypes.Structure):
    _fields_ = [("steps", c_i64), ("buffers", c_i64), ("merged_buffers", c_i64), ("frames_in", c_i64),
                ("samples_out", c_i64), ("admitted", c_i32), ("waiting", c_i32), ("max_admitted", c_i32),
                ("queued", c_i32), ("fixed_bytes", c_i64), ("per_stream_bytes", c_i64)]


class ScError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_LIB = None


def _sig(lib, name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args


def lib():
    """Load the built library (raises if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libstreamconv.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    _sig(L, "sc_plan", c_i32, [P(ScNode), c_i32, P(ScModelInfo)])
    _sig(L, "sc_model_create", c_i32, [P(ScNode), c_i32, c_fp, c_size, c_i32, c_fp, c_u32, c_i32, P(c_vp)])
    _sig(L, "sc_model_create_mixed", c_i32, [P(ScNode), c_i32, c_fp, c_size, P(c_i32), c_fp, c_u32, c_i32,
                                              P(c_vp)])
    _sig(L, "sc_model_info_get", c_i32, [c_vp, P(ScModelInfo)])
    _sig(L, "sc_model_n_layers", c_i32, [c_vp])
    _sig(L, "sc_model_reserve", c_i32, [c_vp, c_i64])
    _sig(L, "sc_model_enable_graph", c_i32, [c_vp, c_i32])
    _sig(L, "sc_stream_state_bytes", c_i64, [c_vp])
    _sig(L, "stream_export", c_i32, [c_vp, c_vp, c_i64])
    _sig(L, "stream_import", c_i32, [c_vp, c_vp, c_i64])
    _sig(L, "sc_model_set_act_scales", c_i32, [c_vp, c_fp])
    _sig(L, "sc_model_read_amax", c_i32, [c_vp, c_fp, c_i32])
    _sig(L, "sc_model_enable_amax", c_i32, [c_vp, c_i32])
    _sig(L, "sc_model_calibrated_scales", c_i32, [c_vp, c_fp])
    _sig(L, "sc_model_destroy", None, [c_vp])
    _sig(L, "stream_create", c_i32, [c_vp, c_i32, c_u32, c_vp, P(c_vp)])
    _sig(L, "stream_process", c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp])
    _sig(L, "stream_process_noalloc", c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp])
    _sig(L, "sc_offline_batch", c_i32, [c_vp, c_i32, P(c_vp), P(c_i32), P(c_vp), c_vp])
    _sig(L, "sc_ola_process", c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp])
    _sig(L, "stream_reset", c_i32, [c_vp, c_vp])
    _sig(L, "stream_position", c_i64, [c_vp])
    _sig(L, "stream_destroy", None, [c_vp])
    _sig(L, "sc_process_batch", c_i32, [c_vp, c_i32, P(c_vp), P(c_vp), P(c_i32), P(c_vp), c_vp])
    _sig(L, "sc_last_error", ctypes.c_char_p, [])
    _sig(L, "sc_model_profile", c_i32, [c_vp, c_i32])
    _sig(L, "sc_model_profile_read", c_i32, [c_vp, P(ScOpProfile), c_i32, P(c_i32)])
    _sig(L, "sc_server_create", c_i32, [c_vp, P(ScServerConfig), P(c_vp)])
    _sig(L, "sc_server_submit", c_i32, [c_vp, c_i64, c_fp, c_i32, P(c_i64)])
    _sig(L, "sc_server_poll", c_i32, [c_vp, c_i64, c_fp, c_i64, P(ctypes.c_double)])
    _sig(L, "sc_server_close_stream", c_i32, [c_vp, c_i64])
    _sig(L, "sc_server_drain", c_i32, [c_vp])
    _sig(L, "sc_server_stats_get", c_i32, [c_vp, P(ScServerStats)])
    _sig(L, "sc_server_destroy", None, [c_vp])
    _sig(L, "sc_server_submit_batch", c_i32, [c_vp, c_i32, P(c_i64), P(c_vp), P(c_i32), c_u32, P(c_i64)])
    _sig(L, "sc_server_latencies", c_i32, [c_vp, P(c_i64), P(ctypes.c_double), c_i64, P(c_i64)])
    _LIB = L
    return L


def check(status):
    if status != SC_OK:
        msg = lib().sc_last_error()
        raise ScError(status, msg.decode() if msg else "")
    return status


def nodes_array(model):
    """Marshal a node-list model (dicts) into a ScNode array."""
    arr = (ScNode * len(model["nodes"]))()
    for i, nd in enumerate(model["nodes"]):
        a = arr[i]
        a.op = OPS[nd["op"]]
        a.src = nd.get("src", -1)
        a.src2 = nd.get("src2", -1)
        if nd["op"] == "input":
            a.cout = nd["channels"]
            continue
        if nd["op"] == "add":
            continue
        a.cin, a.cout, a.k, a.stride = nd["cin"], nd["cout"], nd["k"], nd["stride"]
        a.pre_act = nd.get("pre_act", 0)
        a.post_act = nd.get("post_act", 0)
        if nd["op"] == "conv":
            a.dilation, a.pad_l, a.pad_r = nd["dilation"], nd["pad_l"], nd["pad_r"]
        else:
            a.dilation, a.pad_l, a.pad_r = 1, nd["pad"], nd["pad"]
    return arr


def info_dict(info):
    return {f: getattr(info, f) for f, _ in ScModelInfo._fields_}
