"""ctypes declarations for the C ABI in include/iwpp.h (libiwpp.so)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libiwpp.so")

IWPP_OK = 0
IWPP_EINVAL = -1
IWPP_ENOMEM = -2
IWPP_EDEVICE = -3
IWPP_EBUSY = -4

# Every symbol include/iwpp.h declares (checked by the CPU tests).
EXPORTED = (
    "iwpp_version", "iwpp_create", "iwpp_destroy", "iwpp_last_error",
    "iwpp_morph_recon_u8", "iwpp_edt", "iwpp_get_stats", "iwpp_profile_read", "iwpp_run_batch",
    "iwpp_set_options", "iwpp_round_times", "iwpp_server_start", "iwpp_server_submit", "iwpp_server_poll", "iwpp_server_drain",
    "iwpp_server_get_stats", "iwpp_server_stop", "iwpp_batch_graph_create", "iwpp_batch_graph_launch", "iwpp_batch_graph_stats", "iwpp_batch_graph_destroy",
    "iwpp_batch_graph_round_times",
    "iwpp_round_work",
    "iwpp_morph_recon_u8_noalloc",
    "iwpp_morph_recon_erode_u8",
    "iwpp_morph_recon_queue_u8",
    "iwpp_edt_exact",
)
# Size of the static work area of iwpp_morph_recon_u8_noalloc (IWPP_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 32 << 20
IWPP_OP_RECON = 1
IWPP_OP_EDT = 2
IWPP_OP_RECON_ERODE = 3

KERNEL_NAMES = {0: "reset", 1: "mr_seed", 2: "mr_detect", 3: "mr_propagate", 4: "edt_init", 5: "edt_rounds",
                6: "mrq_init", 7: "mrq_propagate", 8: "edt_exact"}
QUEUE_MODES = {"naive": 0, "ballot": 1, "staged": 2}


class Options(ctypes.Structure):
    _fields_ = [
        ("mr_list_capacity", ctypes.c_int64),
        ("mr_max_sweeps", ctypes.c_int32),
        ("persistent_blocks", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("mr_seed_sweeps", ctypes.c_int32),
        ("wg_waves", ctypes.c_int32),
        ("stage_depth", ctypes.c_int32),
        ("mr_seed_strip", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class QueueOptions(ctypes.Structure):
    _fields_ = [
        ("append_mode", ctypes.c_int32),
        ("seed_sweeps", ctypes.c_int32),
        ("capacity", ctypes.c_int64),
        ("reserved", ctypes.c_int32 * 4),
    ]


class ServerOptions(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_int64),
        ("scratch_bytes", ctypes.c_int64),
        ("max_inflight", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("resident", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 5),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "batches", "max_batch_jobs",
                                              "peak_bytes", "admitted_now", "queued_now")] + [
        ("reserved", ctypes.c_int64 * 4)]


JOB_QUEUED, JOB_ADMITTED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3, 4


class Job(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("conn", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("in0", ctypes.c_void_p),
        ("in1", ctypes.c_void_p),
        ("out0", ctypes.c_void_p),
        ("out1", ctypes.c_void_p),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("ms", ctypes.c_float)]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("seeds", ctypes.c_int64),
        ("items", ctypes.c_int64),
        ("sweeps", ctypes.c_int64),
        ("rounds", ctypes.c_int64),
        ("updates", ctypes.c_int64),
        ("overflow_restarts", ctypes.c_int64),
        ("reserved", ctypes.c_int64 * 6),
    ]


_lib = None


def load():
    """Load libiwpp.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1209_3314_amd.build` "
            "(the GPU library has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.iwpp_version.argtypes = []
    lib.iwpp_version.restype = i32
    lib.iwpp_create.argtypes = [i32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.iwpp_create.restype = i32
    lib.iwpp_destroy.argtypes = [vp]
    lib.iwpp_destroy.restype = None
    lib.iwpp_last_error.argtypes = [vp]
    lib.iwpp_last_error.restype = ctypes.c_char_p
    lib.iwpp_morph_recon_u8.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp]
    lib.iwpp_morph_recon_u8.restype = i32
    lib.iwpp_morph_recon_u8_noalloc.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp]
    lib.iwpp_morph_recon_erode_u8.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp]
    lib.iwpp_morph_recon_erode_u8.restype = i32
    lib.iwpp_morph_recon_queue_u8.argtypes = [vp, vp, vp, vp, i32, i32, i32, ctypes.POINTER(QueueOptions), vp]
    lib.iwpp_morph_recon_queue_u8.restype = i32
    lib.iwpp_edt_exact.argtypes = [vp, vp, vp, vp, i32, i32, vp]
    lib.iwpp_edt_exact.restype = i32
    lib.iwpp_morph_recon_u8_noalloc.restype = i32
    lib.iwpp_edt.argtypes = [vp, vp, vp, vp, i32, i32, i32, vp]
    lib.iwpp_edt.restype = i32
    lib.iwpp_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.iwpp_get_stats.restype = i32
    lib.iwpp_run_batch.argtypes = [vp, ctypes.POINTER(Job), i32, vp]
    lib.iwpp_run_batch.restype = i32
    lib.iwpp_server_start.argtypes = [vp, ctypes.POINTER(ServerOptions), ctypes.POINTER(vp)]
    lib.iwpp_server_start.restype = i32
    lib.iwpp_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.c_int64, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.iwpp_server_submit.restype = i32
    lib.iwpp_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.iwpp_server_poll.restype = i32
    lib.iwpp_server_drain.argtypes = [vp, ctypes.c_int64]
    lib.iwpp_server_drain.restype = i32
    lib.iwpp_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.iwpp_server_get_stats.restype = i32
    lib.iwpp_server_stop.argtypes = [vp]
    lib.iwpp_server_stop.restype = i32
    lib.iwpp_round_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
    lib.iwpp_round_times.restype = i32
    lib.iwpp_round_work.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), i32,
                                    ctypes.POINTER(i32)]
    lib.iwpp_round_work.restype = i32
    lib.iwpp_set_options.argtypes = [vp, ctypes.POINTER(Options)]
    lib.iwpp_set_options.restype = i32
    lib.iwpp_batch_graph_create.argtypes = [vp, ctypes.POINTER(Job), i32, ctypes.POINTER(vp)]
    lib.iwpp_batch_graph_create.restype = i32
    lib.iwpp_batch_graph_launch.argtypes = [vp, vp]
    lib.iwpp_batch_graph_launch.restype = i32
    lib.iwpp_batch_graph_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.iwpp_batch_graph_stats.restype = i32
    lib.iwpp_batch_graph_round_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32, ctypes.POINTER(i32)]
    lib.iwpp_batch_graph_round_times.restype = i32
    lib.iwpp_batch_graph_destroy.argtypes = [vp]
    lib.iwpp_batch_graph_destroy.restype = None
    lib.iwpp_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
    lib.iwpp_profile_read.restype = i32
    _lib = lib
    return lib
