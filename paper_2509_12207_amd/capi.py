"""ctypes binding of libug (include/ug.h): argument marshalling only.

Every computation happens in the library (gate thread, policy, gfx950
kernels).  The library is built in-tree by ``paper_2509_12207_amd.build``;
loading fails loudly if it is missing.
"""

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libug.so")

ABI_VERSION = 7

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ETIMEDOUT, ESTATE, ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
POLICY_FIFO, POLICY_URGENCY = 0, 1
F_BIND, F_DELAY, F_BATCH, F_CALIBRATE, F_ADMIT, F_EXIT, F_NO_OVERLAP = 1, 2, 4, 8, 16, 32, 64
F_GRAPH = 128
F_PLACE = 256
F_CPU_PRIO = 512
F_FUSE = 1024

KEY_URGENCY, KEY_EDF, KEY_SJF, KEY_HRRN, KEY_LCUF, KEY_SAEDF, KEY_EQDF = 0, 1, 2, 3, 4, 5, 6
KEYS = {"urgency": KEY_URGENCY, "edf": KEY_EDF, "sjf": KEY_SJF, "hrrn": KEY_HRRN, "lcuf": KEY_LCUF,
        "saedf": KEY_SAEDF, "eqdf": KEY_EQDF}

OP_GEMM_F32 = 1
OP_BIAS_RELU_F32 = 2
OP_CONV3X3_F32 = 3
OP_ROWSUM_F32 = 4
OP_SOFTMAX_F32 = 5
OP_VOXEL_F32 = 6
OP_GEMM_FP8 = 7
OP_GEMM_BF16 = 8
OP_VECADD_F32 = 9
OP_CONV3X3_BF16 = 10
OP_UPLOAD_H2D = 11
OP_ACCUM_I32 = 12
OP_NAMES = {OP_GEMM_F32: "gemm", OP_BIAS_RELU_F32: "bias_relu", OP_CONV3X3_F32: "conv3x3",
            OP_ROWSUM_F32: "rowsum", OP_SOFTMAX_F32: "softmax", OP_VOXEL_F32: "voxel",
            OP_GEMM_FP8: "gemm_fp8", OP_GEMM_BF16: "gemm_bf16", OP_VECADD_F32: "vecadd",
            OP_CONV3X3_BF16: "conv3x3_bf16", OP_UPLOAD_H2D: "upload", OP_ACCUM_I32: "accum_i32"}
OP_IDS = {v: k for k, v in OP_NAMES.items()}

REC_INSTANT, REC_ARRIVE, REC_EVDONE, REC_COMPLETE = 1, 2, 3, 4
REC_TSTART, REC_BIND, REC_HOLD, REC_EVREC, REC_LAUNCH, REC_EXIT, REC_DIMS = 5, 6, 7, 8, 9, 10, 11
REC_CPU = 12

EXPORTED = [
    "ug_config_default", "ug_now_ns", "ug_status_str", "ug_create", "ug_destroy",
    "ug_last_error", "ug_chain_register", "ug_kernel_set_estimate", "ug_kernel_get_estimate",
    "ug_profile", "ug_set_threshold", "ug_set_flags", "ug_start", "ug_frame_submit",
    "ug_poll_complete", "ug_drain", "ug_stop", "ug_get_stats", "ug_trace_read",
    "ug_calibration_read", "ug_calibration_threshold", "ug_get_metrics", "ug_replay_instant",
    "ug_kernel_launch", "ug_kernel_util", "ug_kernel_workspace", "ug_kernel_launch_ws",
    "ug_frame_submit_dims", "ug_chain_set_footprint", "ug_streams_needed", "ug_attach_streams",
    "ug_kernel_launch_noalloc", "ug_kernel_set_profile", "ug_kernel_get_profile",
    "ug_tails_open", "ug_tails_publish", "ug_tails_set_key", "ug_tails_pause", "ug_tails_kick",
    "ug_tails_finished", "ug_tails_log", "ug_tails_close", "ug_kernel_launch_signal",
    "ug_chain_tails", "ug_launch_cost", "ug_tile_variants", "ug_tile_set", "ug_tile_clear",
    "ug_tile_get", "ug_tile_load", "ug_kernel_launch_variant", "ug_graph_prepare",
    "ug_tails_stats", "ug_fuse_stats",
]

# the executor's statistics (ug_tails_stats / ug_fuse_stats), in order
FUSE_STATS = ("rounds", "round_ticks", "items", "wait_ticks", "queue_ticks", "serve_ticks",
              "tiles")


class Kernel(C.Structure):
    _fields_ = [("op", C.c_int32), ("in_", C.c_int32 * 3), ("out", C.c_int32 * 4),
                ("shape", C.c_int64 * 4), ("fparam", C.c_float * 4), ("est_ns", C.c_int64),
                ("util", C.c_float), ("frame_dim", C.c_int32), ("frame_shift", C.c_int32),
                ("pad0", C.c_int32)]


class Task(C.Structure):
    _fields_ = [("kernels", C.POINTER(Kernel)), ("n_kernels", C.c_uint32),
                ("pad0", C.c_uint32), ("cpu_ns", C.c_int64)]


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("policy", C.c_int32), ("flags", C.c_uint32),
                ("device", C.c_int32), ("delta_eval_ns", C.c_int64),
                ("delay_poll_ns", C.c_int64), ("util_exempt", C.c_float),
                ("n_levels", C.c_int32), ("lanes", C.c_int32 * 8), ("th_slack_ns", C.c_int64),
                ("idle_sleep_ns", C.c_int64), ("queue_capacity", C.c_uint32),
                ("trace_capacity", C.c_uint32), ("calib_period_ns", C.c_int64),
                ("admit_tasks", C.c_int64), ("hbm_budget_bytes", C.c_uint64),
                ("order_key", C.c_int32), ("est_noise_permille", C.c_int32),
                ("noise_seed", C.c_uint64), ("max_hold_ns", C.c_int64),
                ("own_streams", C.c_int32), ("cpu_cores", C.c_int32),
                ("fuse_workers", C.c_uint32), ("pad1", C.c_int32), ("fuse_idle_ns", C.c_int64),
                ("tile_table", C.c_char_p)]


class Completion(C.Structure):
    _fields_ = [("chain", C.c_uint32), ("pad0", C.c_uint32), ("frame", C.c_uint64),
                ("t_arr_ns", C.c_int64), ("t_done_ns", C.c_int64), ("latency_ns", C.c_int64),
                ("missed", C.c_int32), ("n_holds", C.c_int32), ("n_batches", C.c_int32),
                ("exited", C.c_int32)]


class Record(C.Structure):
    _fields_ = [("type", C.c_int32), ("chain", C.c_int32), ("frame", C.c_int64),
                ("task", C.c_int32), ("kernel", C.c_int32), ("a", C.c_int32), ("b", C.c_int32),
                ("t", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("frames_submitted", C.c_uint64), ("frames_completed", C.c_uint64),
                ("frames_missed", C.c_uint64), ("launches", C.c_uint64), ("holds", C.c_uint64),
                ("batches", C.c_uint64), ("instants", C.c_uint64), ("collisions", C.c_uint64),
                ("decide_ns", C.c_int64), ("launch_ns", C.c_int64),
                ("trace_records", C.c_uint64), ("trace_dropped", C.c_uint64),
                ("frames_deferred", C.c_uint64), ("hbm_peak_bytes", C.c_uint64),
                ("tails_fused", C.c_uint64), ("tails_unfused", C.c_uint64),
                ("executor_launches", C.c_uint64), ("collision_hist", C.c_uint64 * 8)]


class Tail(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("bias", C.c_void_p), ("sm", C.c_void_p),
                ("rs", C.c_void_p), ("counter", C.c_void_p), ("counter_target", C.c_uint32),
                ("rows", C.c_uint32), ("cols", C.c_uint32), ("axis", C.c_uint32)]


class Metrics(C.Structure):
    _fields_ = [("frames", C.c_uint64), ("missed", C.c_uint64), ("miss_ratio", C.c_double),
                ("p50_ns", C.c_int64), ("p99_ns", C.c_int64), ("max_ns", C.c_int64),
                ("mean_ns", C.c_double), ("n_chains", C.c_uint32), ("pad0", C.c_uint32)]


RECORD_DTYPE = np.dtype([("type", np.int32), ("chain", np.int32), ("frame", np.int64),
                         ("task", np.int32), ("kernel", np.int32), ("a", np.int32),
                         ("b", np.int32), ("t", np.int64)])
COMPLETION_DTYPE = np.dtype([("chain", np.uint32), ("pad0", np.uint32), ("frame", np.uint64),
                             ("t_arr_ns", np.int64), ("t_done_ns", np.int64),
                             ("latency_ns", np.int64), ("missed", np.int32),
                             ("n_holds", np.int32), ("n_batches", np.int32), ("exited", np.int32)])

_lib = None


class UgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libug error {status}: {msg}")
        self.status = status


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "__graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.ug_config_default.argtypes = [C.POINTER(Config)]
        L.ug_config_default.restype = None
        L.ug_now_ns.restype = C.c_int64
        L.ug_status_str.argtypes = [C.c_int32]
        L.ug_status_str.restype = C.c_char_p
        L.ug_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.ug_destroy.argtypes = [vp]
        L.ug_destroy.restype = None
        L.ug_last_error.argtypes = [vp]
        L.ug_last_error.restype = C.c_char_p
        L.ug_chain_register.argtypes = [vp, C.c_int64, C.c_int64, C.POINTER(Task), C.c_uint32,
                                        C.c_uint32, C.POINTER(C.c_uint32)]
        L.ug_kernel_set_estimate.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_int64, C.c_float]
        L.ug_kernel_get_estimate.argtypes = [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64),
                                             C.POINTER(C.c_float)]
        L.ug_profile.argtypes = [vp, C.c_uint32, C.POINTER(vp), C.c_uint32, C.c_uint32, C.c_uint32]
        L.ug_set_threshold.argtypes = [vp, C.c_int64]
        L.ug_set_flags.argtypes = [vp, C.c_int32, C.c_uint32]
        L.ug_start.argtypes = [vp]
        L.ug_frame_submit.argtypes = [vp, C.c_uint32, C.c_int64, C.POINTER(vp), C.c_uint32,
                                      C.POINTER(C.c_uint64)]
        L.ug_poll_complete.argtypes = [vp, C.POINTER(Completion), C.c_uint32]
        L.ug_drain.argtypes = [vp, C.c_int64]
        L.ug_stop.argtypes = [vp]
        L.ug_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.ug_trace_read.argtypes = [vp, C.POINTER(Record), C.c_uint32]
        L.ug_calibration_read.argtypes = [vp, C.POINTER(C.c_int64), C.c_uint32]
        L.ug_calibration_threshold.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
        L.ug_get_metrics.argtypes = [vp, C.POINTER(Metrics)]
        L.ug_replay_instant.argtypes = [vp, C.c_int64, C.POINTER(Record), C.c_uint32,
                                        C.POINTER(Record), C.c_uint32, C.POINTER(C.c_uint32)]
        L.ug_kernel_launch.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32, vp]
        L.ug_kernel_util.argtypes = [C.POINTER(Kernel), C.c_int32, C.POINTER(C.c_float)]
        L.ug_kernel_workspace.argtypes = [C.POINTER(Kernel), C.POINTER(C.c_uint64)]
        L.ug_kernel_launch_ws.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32, vp,
                                          C.c_uint64, vp]
        L.ug_frame_submit_dims.argtypes = [vp, C.c_uint32, C.c_int64, C.POINTER(vp), C.c_uint32,
                                           C.POINTER(C.c_int64), C.c_uint32,
                                           C.POINTER(C.c_uint64)]
        L.ug_chain_set_footprint.argtypes = [vp, C.c_uint32, C.c_uint64]
        L.ug_streams_needed.argtypes = [vp, C.POINTER(C.c_uint32)]
        L.ug_attach_streams.argtypes = [vp, C.POINTER(vp), C.c_uint32]
        L.ug_kernel_launch_noalloc.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32, vp]
        L.ug_kernel_set_profile.argtypes = [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64),
                                            C.POINTER(C.c_int64), C.c_uint32]
        L.ug_kernel_get_profile.argtypes = [vp, C.c_uint32, C.c_uint32, C.POINTER(C.c_int64),
                                            C.POINTER(C.c_int64), C.c_uint32,
                                            C.POINTER(C.c_uint32)]
        L.ug_tails_open.argtypes = [C.c_int32, C.c_uint32, C.c_int64, C.c_uint32, C.POINTER(vp)]
        L.ug_tails_publish.argtypes = [vp, C.POINTER(Tail), C.c_uint64, C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint64)]
        L.ug_tails_set_key.argtypes = [vp, C.c_uint32, C.c_uint64]
        L.ug_tails_pause.argtypes = [vp, C.c_int32]
        L.ug_tails_kick.argtypes = [vp]
        L.ug_tails_finished.argtypes = [vp, C.c_uint32, C.c_uint64]
        L.ug_tails_log.argtypes = [vp, C.POINTER(C.c_uint64), C.c_uint32]
        L.ug_tails_stats.argtypes = [vp, C.POINTER(C.c_uint64), C.c_uint32]
        L.ug_fuse_stats.argtypes = [vp, C.POINTER(C.c_uint64), C.c_uint32]
        L.ug_tails_close.argtypes = [vp]
        L.ug_kernel_launch_signal.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32, vp,
                                              C.POINTER(C.c_uint32), vp]
        L.ug_chain_tails.argtypes = [vp, C.c_uint32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.c_uint32]
        L.ug_launch_cost.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32, C.c_uint32, vp,
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ug_graph_prepare.argtypes = [vp, C.c_uint32, C.POINTER(vp), C.c_uint32,
                                       C.POINTER(C.c_int64), C.c_uint32]
        L.ug_tile_variants.argtypes = [C.c_int32]
        L.ug_tile_set.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.c_int32]
        L.ug_tile_clear.argtypes = []
        L.ug_tile_get.argtypes = [C.POINTER(Kernel)]
        L.ug_tile_load.argtypes = [C.c_char_p, C.POINTER(C.c_uint32)]
        L.ug_kernel_launch_variant.argtypes = [C.POINTER(Kernel), C.POINTER(vp), C.c_uint32,
                                               C.c_int32, vp]
        for name in ("ug_create", "ug_chain_register", "ug_kernel_set_estimate",
                     "ug_kernel_get_estimate", "ug_profile", "ug_set_threshold", "ug_set_flags",
                     "ug_start", "ug_frame_submit", "ug_poll_complete", "ug_drain", "ug_stop",
                     "ug_get_stats", "ug_trace_read", "ug_calibration_read",
                     "ug_calibration_threshold", "ug_get_metrics", "ug_replay_instant",
                     "ug_kernel_launch", "ug_kernel_util", "ug_frame_submit_dims",
                     "ug_chain_set_footprint", "ug_streams_needed", "ug_attach_streams",
                     "ug_kernel_launch_noalloc", "ug_kernel_set_profile",
                     "ug_kernel_get_profile", "ug_tails_open", "ug_tails_publish",
                     "ug_tails_set_key", "ug_tails_pause", "ug_tails_kick", "ug_tails_finished",
                     "ug_tails_log", "ug_tails_close", "ug_kernel_launch_signal",
                     "ug_chain_tails", "ug_launch_cost", "ug_tile_variants", "ug_tile_set",
                     "ug_tile_clear", "ug_tile_get", "ug_tile_load",
                     "ug_kernel_launch_variant", "ug_graph_prepare", "ug_tails_stats",
                     "ug_fuse_stats"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def status_str(s):
    return lib().ug_status_str(s).decode()


# --------------------------------------------------------------------------
# descriptors
# --------------------------------------------------------------------------
def kernel_struct(k):
    """Kernel descriptor dict -> ug_kernel.

    dict keys: op (name or id), shape (<= 4 ints), in (<= 3 slots), out (<= 4
    slots), fparam (<= 4 floats), est_ns (int, default 0), util (float,
    default -1 = derive from the launch shape), frame_dim (int, default 0 =
    fixed shape; d >= 1: a per-frame size, each frame gives its own value as
    dims[d - 1]), frame_shift (int, default 0).
    """
    s = Kernel()
    op = k["op"]
    s.op = OP_IDS[op] if isinstance(op, str) else int(op)
    for i in range(3):
        s.in_[i] = -1
    for i in range(4):
        s.out[i] = -1
    for i, v in enumerate(k.get("in", ())):
        s.in_[i] = int(v)
    for i, v in enumerate(k.get("out", ())):
        s.out[i] = int(v)
    for i, v in enumerate(k.get("shape", ())):
        s.shape[i] = int(v)
    for i, v in enumerate(k.get("fparam", ())):
        s.fparam[i] = float(v)
    s.est_ns = int(k.get("est_ns", 0))
    s.util = float(k.get("util", -1.0))
    s.frame_dim = int(k.get("frame_dim", 0))
    s.frame_shift = int(k.get("frame_shift", 0))
    return s


def pointer_array(ptrs):
    arr = (C.c_void_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = int(p)
    return arr


def kernel_launch(k, ptrs, stream=None):
    """Launch one kernel on a HIP stream (an int handle, or None for the default)."""
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    st = lib().ug_kernel_launch(C.byref(ks), arr, len(ptrs), C.c_void_p(stream or 0))
    if st != OK:
        raise UgError(st, f"ug_kernel_launch({OP_NAMES.get(ks.op, ks.op)})")


STATIC_SCRATCH_BYTES = 64 << 20   # UG_STATIC_SCRATCH_BYTES


def kernel_launch_noalloc(k, ptrs, stream=None):
    """Launch one kernel without allocating (static device workspace)."""
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    st = lib().ug_kernel_launch_noalloc(C.byref(ks), arr, len(ptrs), C.c_void_p(stream or 0))
    if st != OK:
        raise UgError(st, f"ug_kernel_launch_noalloc({OP_NAMES.get(ks.op, ks.op)})")


def kernel_workspace(k):
    """Bytes of device workspace kernel ``k`` needs beside its buffers."""
    n = C.c_uint64()
    st = lib().ug_kernel_workspace(C.byref(kernel_struct(k)), C.byref(n))
    if st != OK:
        raise UgError(st, "ug_kernel_workspace")
    return int(n.value)


def kernel_launch_ws(k, ptrs, ws_ptr, ws_bytes, stream=None):
    """Launch one kernel with a caller-owned device workspace."""
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    st = lib().ug_kernel_launch_ws(C.byref(ks), arr, len(ptrs), C.c_void_p(ws_ptr or 0),
                                   ws_bytes, C.c_void_p(stream or 0))
    if st != OK:
        raise UgError(st, f"ug_kernel_launch_ws({OP_NAMES.get(ks.op, ks.op)})")


def kernel_util(k, device=0):
    u = C.c_float()
    st = lib().ug_kernel_util(C.byref(kernel_struct(k)), device, C.byref(u))
    if st != OK:
        raise UgError(st, "ug_kernel_util")
    return float(u.value)


def now_ns():
    return int(lib().ug_now_ns())


def kernel_launch_signal(k, ptrs, counter_ptr, stream=None):
    """Launch a contraction that adds one per finished wavefront to the
    device counter at ``counter_ptr``; returns the final count."""
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    waves = C.c_uint32()
    st = lib().ug_kernel_launch_signal(C.byref(ks), arr, len(ptrs), C.c_void_p(counter_ptr),
                                       C.byref(waves), C.c_void_p(stream or 0))
    if st != OK:
        raise UgError(st, f"ug_kernel_launch_signal({OP_NAMES.get(ks.op, ks.op)})")
    return int(waves.value)


def tile_variants(op):
    return int(lib().ug_tile_variants(OP_IDS[op] if isinstance(op, str) else int(op)))


def tile_set(op, shape, variant):
    sh = (C.c_int64 * 4)(*(list(shape) + [0] * (4 - len(shape))))
    st = lib().ug_tile_set(OP_IDS[op] if isinstance(op, str) else int(op), sh, int(variant))
    if st != OK:
        raise UgError(st, "ug_tile_set")


def tile_clear():
    lib().ug_tile_clear()


def tile_get(k):
    return int(lib().ug_tile_get(C.byref(kernel_struct(k))))


def tile_load(path):
    n = C.c_uint32()
    st = lib().ug_tile_load(os.fsencode(path), C.byref(n))
    if st != OK:
        raise UgError(st, f"ug_tile_load({path})")
    return int(n.value)


def kernel_launch_variant(k, ptrs, variant, stream=None):
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    st = lib().ug_kernel_launch_variant(C.byref(ks), arr, len(ptrs), int(variant),
                                        C.c_void_p(stream or 0))
    if st != OK:
        raise UgError(st, f"ug_kernel_launch_variant({OP_NAMES.get(ks.op, ks.op)}, {variant})")


def launch_cost(k, ptrs, n=2000, stream=None):
    """Raw launch loop of n kernels: (host ns per launch call, device ns per
    kernel)."""
    ks = kernel_struct(k)
    arr = pointer_array(ptrs)
    h, g = C.c_int64(), C.c_int64()
    st = lib().ug_launch_cost(C.byref(ks), arr, len(ptrs), n, C.c_void_p(stream or 0),
                              C.byref(h), C.byref(g))
    if st != OK:
        raise UgError(st, "ug_launch_cost")
    return int(h.value), int(g.value)


class TailQueue:
    """The tail executor's queue (ug_tails_*), driven directly."""

    def __init__(self, device=0, workers=64, idle_ns=500_000, log_cap=0):
        h = C.c_void_p()
        st = lib().ug_tails_open(device, workers, idle_ns, log_cap, C.byref(h))
        if st != OK:
            raise UgError(st, "ug_tails_open")
        self.h = h

    def publish(self, x, y, bias, rows, cols, axis, key, sm=0, rs=0, counter=0, target=0):
        t = Tail(x, y, bias, sm or None, rs or None, counter or None, target, rows, cols, axis)
        slot, pub = C.c_uint32(), C.c_uint64()
        st = lib().ug_tails_publish(self.h, C.byref(t), key, C.byref(slot), C.byref(pub))
        if st != OK:
            raise UgError(st, "ug_tails_publish")
        return int(slot.value), int(pub.value)

    def set_key(self, slot, key):
        st = lib().ug_tails_set_key(self.h, slot, key)
        if st != OK:
            raise UgError(st, "ug_tails_set_key")

    def pause(self, on):
        st = lib().ug_tails_pause(self.h, 1 if on else 0)
        if st != OK:
            raise UgError(st, "ug_tails_pause")

    def kick(self):
        st = lib().ug_tails_kick(self.h)
        if st != OK:
            raise UgError(st, "ug_tails_kick")

    def finished(self, slot, pub):
        r = lib().ug_tails_finished(self.h, slot, pub)
        if r < 0:
            raise UgError(r, "ug_tails_finished")
        return bool(r)

    def log(self, cap=8192):
        out = (C.c_uint64 * max(1, cap))()
        n = lib().ug_tails_log(self.h, out, cap)
        if n < 0:
            raise UgError(n, "ug_tails_log")
        return [int(out[i]) for i in range(n)]

    def stats(self):
        out = (C.c_uint64 * len(FUSE_STATS))()
        st = lib().ug_tails_stats(self.h, out, len(FUSE_STATS))
        if st != OK:
            raise UgError(st, "ug_tails_stats")
        return dict(zip(FUSE_STATS, (int(v) for v in out)))

    def close(self):
        if self.h:
            st = lib().ug_tails_close(self.h)
            self.h = None
            if st != OK:
                raise UgError(st, "ug_tails_close")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# context
# --------------------------------------------------------------------------
class Gate:
    """One libug context.

    ``policy``: "urgency" or "fifo".  Keyword arguments override the fields
    of ug_config (``lanes`` takes a list, one entry per level).  FIFO launch
    takes no flags unless given (in particular no queue placement: the
    baseline keeps HIP's own stream-to-queue mapping).

    The stream pool comes from torch: ``start`` attaches default-priority
    ``torch.cuda.Stream`` objects (kept alive by this object) unless streams
    were attached before or the library owns its streams (``own_streams=1``).
    torch hands out streams from a fixed pool of 32 per device, so FIFO
    launch, which needs one stream per task of every chain, lets the
    library create its own unless given ``own_streams=0`` (then attach
    distinct streams before ``start``).
    """

    def __init__(self, policy="urgency", device=0, **kw):
        L = lib()
        cfg = Config()
        L.ug_config_default(C.byref(cfg))
        cfg.policy = POLICY_URGENCY if policy == "urgency" else POLICY_FIFO
        cfg.device = device
        if cfg.policy == POLICY_FIFO:
            cfg.flags = 0
            cfg.own_streams = 1
        lanes = kw.pop("lanes", None)
        key = kw.pop("order_key", None)
        if key is not None:
            cfg.order_key = KEYS[key] if isinstance(key, str) else int(key)
        if lanes is not None:
            cfg.n_levels = len(lanes)
            for i in range(8):
                cfg.lanes[i] = lanes[i] if i < len(lanes) else 0
        for key, v in kw.items():
            if key == "tile_table" and isinstance(v, str):
                v = os.fsencode(v)
            setattr(cfg, key, v)
        self.cfg = cfg
        h = C.c_void_p()
        st = L.ug_create(C.byref(cfg), C.byref(h))
        if st != OK:
            raise UgError(st, "ug_create: " + L.ug_last_error(None).decode())
        self.h = h
        self._keep = []
        self._streams = None      # torch streams lent to the library

    def _check(self, st, what):
        if st != OK:
            msg = lib().ug_last_error(self.h).decode() if self.h else ""
            raise UgError(st, f"{what}: {msg}")

    def close(self):
        if self.h:
            lib().ug_destroy(self.h)     # drains the streams before returning
            self.h = None
        self._streams = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register_chain(self, period_ns, deadline_ns, tasks, n_buffers):
        """tasks: list of {"cpu_ns": int, "kernels": [kernel dicts]}."""
        arrays = []
        tarr = (Task * len(tasks))()
        for j, t in enumerate(tasks):
            ks = (Kernel * len(t["kernels"]))(*[kernel_struct(k) for k in t["kernels"]])
            arrays.append(ks)
            tarr[j].kernels = C.cast(ks, C.POINTER(Kernel))
            tarr[j].n_kernels = len(t["kernels"])
            tarr[j].cpu_ns = int(t.get("cpu_ns", 0))
        cid = C.c_uint32()
        st = lib().ug_chain_register(self.h, int(period_ns), int(deadline_ns), tarr, len(tasks),
                                     int(n_buffers), C.byref(cid))
        self._check(st, "ug_chain_register")
        return int(cid.value)

    def prepare_graphs(self, chain, ptrs, dims=None):
        """Capture the chain's task graphs for one buffer set before start."""
        arr = pointer_array(ptrs)
        d = (C.c_int64 * max(1, len(dims or [])))(*(dims or []))
        self._check(lib().ug_graph_prepare(self.h, chain, arr, len(ptrs), d, len(dims or [])),
                    "ug_graph_prepare")

    def chain_tails(self, chain, cap=4096):
        """(first, end) kernel ranges of the chain's tails that UG_F_FUSE fuses."""
        f = (C.c_int32 * max(1, cap))()
        e = (C.c_int32 * max(1, cap))()
        n = lib().ug_chain_tails(self.h, chain, f, e, cap)
        self._check(min(n, 0), "ug_chain_tails")
        return [(int(f[i]), int(e[i])) for i in range(n)]

    def set_estimate(self, chain, kernel, est_ns, util=-1.0):
        self._check(lib().ug_kernel_set_estimate(self.h, chain, kernel, int(est_ns), float(util)),
                    "ug_kernel_set_estimate")

    def get_estimate(self, chain, kernel):
        e, u = C.c_int64(), C.c_float()
        self._check(lib().ug_kernel_get_estimate(self.h, chain, kernel, C.byref(e), C.byref(u)),
                    "ug_kernel_get_estimate")
        return int(e.value), float(u.value)

    def set_profile(self, chain, kernel, points):
        """Profile points [(v, E_ns), ...] of a kernel with a per-frame size."""
        n = len(points)
        v = (C.c_int64 * max(1, n))(*[int(p[0]) for p in points])
        e = (C.c_int64 * max(1, n))(*[int(p[1]) for p in points])
        self._check(lib().ug_kernel_set_profile(self.h, chain, kernel, v, e, n),
                    "ug_kernel_set_profile")

    def get_profile(self, chain, kernel, cap=16):
        v, e, n = (C.c_int64 * cap)(), (C.c_int64 * cap)(), C.c_uint32()
        self._check(lib().ug_kernel_get_profile(self.h, chain, kernel, v, e, cap, C.byref(n)),
                    "ug_kernel_get_profile")
        return [(int(v[i]), int(e[i])) for i in range(min(cap, n.value))]

    def profile(self, chain, ptrs, warmup=3, reps=10):
        arr = pointer_array(ptrs)
        self._check(lib().ug_profile(self.h, chain, arr, len(ptrs), warmup, reps), "ug_profile")

    def set_threshold(self, th_slack_ns):
        self._check(lib().ug_set_threshold(self.h, int(th_slack_ns)), "ug_set_threshold")

    def set_flags(self, flags):
        self._check(lib().ug_set_flags(self.h, self.cfg.policy, int(flags)), "ug_set_flags")
        self.cfg.flags = flags

    def streams_needed(self):
        n = C.c_uint32()
        self._check(lib().ug_streams_needed(self.h, C.byref(n)), "ug_streams_needed")
        return int(n.value)

    def attach_streams(self, streams=None):
        """Lend the library its stream pool: ``streams`` is a list of
        ``torch.cuda.Stream`` (default: new ones at the default priority, as
        many as ``ug_streams_needed``).  They stay referenced here until
        ``close``."""
        if streams is None:
            import torch
            dev = torch.device("cuda", self.cfg.device)
            n = self.streams_needed()
            if n > 32:
                raise ValueError(f"{n} streams: more than torch's pool of 32 distinct streams "
                                 "(create the context with own_streams=1)")
            streams = [torch.cuda.Stream(device=dev) for _ in range(n)]
        arr = pointer_array([s.cuda_stream for s in streams])
        self._check(lib().ug_attach_streams(self.h, arr, len(streams)), "ug_attach_streams")
        self._streams = list(streams)

    def start(self):
        if self._streams is None and not self.cfg.own_streams and self.cfg.device >= 0:
            self.attach_streams()
        self._check(lib().ug_start(self.h), "ug_start")

    def stop(self):
        self._check(lib().ug_stop(self.h), "ug_stop")

    def submit(self, chain, t_arr_ns, ptrs, dims=None):
        """Frame index, or None when refused with UG_EAGAIN (queue full or
        HBM budget).  ``dims``: per-frame sizes (kernels with frame_dim)."""
        arr = pointer_array(ptrs)
        f = C.c_uint64()
        if dims is None:
            st = lib().ug_frame_submit(self.h, chain, int(t_arr_ns), arr, len(ptrs), C.byref(f))
        else:
            d = (C.c_int64 * max(1, len(dims)))(*[int(x) for x in dims])
            st = lib().ug_frame_submit_dims(self.h, chain, int(t_arr_ns), arr, len(ptrs), d,
                                            len(dims), C.byref(f))
        if st == EAGAIN:
            return None
        self._check(st, "ug_frame_submit")
        return int(f.value)

    def set_footprint(self, chain, nbytes):
        self._check(lib().ug_chain_set_footprint(self.h, chain, int(nbytes)),
                    "ug_chain_set_footprint")

    def poll(self, cap=4096):
        buf = (Completion * cap)()
        n = lib().ug_poll_complete(self.h, buf, cap)
        if n < 0:
            self._check(n, "ug_poll_complete")
        out = np.frombuffer(bytes(buf)[: n * C.sizeof(Completion)], dtype=COMPLETION_DTYPE)
        return out.copy()

    def drain(self, timeout_s=60.0):
        self._check(lib().ug_drain(self.h, int(timeout_s * 1e9)), "ug_drain")

    def fuse_stats(self):
        out = (C.c_uint64 * len(FUSE_STATS))()
        self._check(lib().ug_fuse_stats(self.h, out, len(FUSE_STATS)), "ug_fuse_stats")
        return dict(zip(FUSE_STATS, (int(v) for v in out)))

    def stats(self):
        s = Stats()
        self._check(lib().ug_get_stats(self.h, C.byref(s)), "ug_get_stats")
        return {f: (list(getattr(s, f)) if f == "collision_hist" else getattr(s, f))
                for f, _ in Stats._fields_}

    def trace(self, cap=1 << 20):
        chunks = []
        while True:
            buf = (Record * cap)()
            n = lib().ug_trace_read(self.h, buf, cap)
            if n < 0:
                self._check(n, "ug_trace_read")
            chunks.append(np.frombuffer(bytes(buf)[: n * C.sizeof(Record)], dtype=RECORD_DTYPE).copy())
            if n < cap:
                break
        return np.concatenate(chunks) if chunks else np.zeros(0, RECORD_DTYPE)

    def calibration_samples(self, cap=1 << 22):
        buf = (C.c_int64 * cap)()
        n = lib().ug_calibration_read(self.h, buf, cap)
        if n < 0:
            self._check(n, "ug_calibration_read")
        return [int(buf[i]) for i in range(n)]

    def calibration_threshold(self, pct=95):
        th = C.c_int64()
        self._check(lib().ug_calibration_threshold(self.h, int(pct), C.byref(th)),
                    "ug_calibration_threshold")
        return int(th.value)

    def metrics(self):
        m = Metrics()
        self._check(lib().ug_get_metrics(self.h, C.byref(m)), "ug_get_metrics")
        return {f: getattr(m, f) for f, _ in Metrics._fields_ if f != "pad0"}

    def replay_instant(self, t, inputs, cap=1 << 16):
        """inputs: numpy RECORD_DTYPE array (ARRIVE / EVDONE records)."""
        n_in = len(inputs)
        inp = (Record * max(1, n_in))()
        if n_in:
            C.memmove(inp, np.ascontiguousarray(inputs, dtype=RECORD_DTYPE).ctypes.data,
                      n_in * C.sizeof(Record))
        out = (Record * cap)()
        n_out = C.c_uint32()
        self._check(lib().ug_replay_instant(self.h, int(t), inp, n_in, out, cap, C.byref(n_out)),
                    "ug_replay_instant")
        return np.frombuffer(bytes(out)[: n_out.value * C.sizeof(Record)], dtype=RECORD_DTYPE).copy()
