"""ctypes declarations of libaesctr.so (mirrors include/aesctr.h).

Argument marshalling only: every step of the cipher runs in the library's
HIP kernels.  Importing this module loads the library and raises if it is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaesctr.so")

AES_OK = 0
AES_EINVAL = -1
AES_ENOMEM = -2
AES_EAGAIN = -3
AES_ERANGE = -4
AES_EDEVICE = -5
AES_ENOTFOUND = -6
AES_ETIMEDOUT = -7
AES_EOVERLAP = -8
AES_ECLOSED = -9
AES_ECANCELED = -10
AES_ETOOBIG = -11
AES_FLAG_SHA256 = 1

AES_VARIANT_AUTO = 0
AES_VARIANT_TTABLE = 1
AES_VARIANT_BITSLICE = 2
AES_VARIANT_VPERM = 3


class aes_sched_t(ctypes.Structure):
    _fields_ = [("rk", ctypes.c_uint32 * 60), ("nr", ctypes.c_int32), ("key_bits", ctypes.c_int32)]


class aes_launch_cfg_t(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("blocks_per_lane", ctypes.c_int32),
                ("wg_size", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("lds_copies", ctypes.c_int32), ("lds_tables", ctypes.c_int32),
                ("wave_groups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class aes_ctr_desc_t(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("len", ctypes.c_uint64),
                ("sched", ctypes.POINTER(aes_sched_t)), ("nonce", ctypes.c_uint8 * 12),
                ("ctr0", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class sha256_desc_t(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("len", ctypes.c_uint64), ("digest", ctypes.c_void_p),
                ("reserved", ctypes.c_uint64)]


class aes_batch_cfg_t(ctypes.Structure):
    _fields_ = [("tile_bytes", ctypes.c_int32), ("wg_size", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("blocks_per_lane", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class aes_engine_cfg_t(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("n_streams", ctypes.c_int32),
                ("max_batch_reqs", ctypes.c_int32), ("max_batch_bytes", ctypes.c_uint64),
                ("key_slots", ctypes.c_int32), ("host_buffers", ctypes.c_int32),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class aes_stats_t(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("bytes_completed", ctypes.c_uint64), ("budget_high_water", ctypes.c_uint64),
                ("queued_now", ctypes.c_uint64), ("inflight_now", ctypes.c_uint64),
                ("mean_batch_reqs", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("p999_us", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("max_us", ctypes.c_double),
                ("key_hits", ctypes.c_uint64), ("key_misses", ctypes.c_uint64)]


# Every exported name and its (restype, argtypes).
SIGNATURES = {
    "aes_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "aes_last_device_error": (ctypes.c_char_p, []),
    "aes_expand_key": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(aes_sched_t)]),
    "aes_ctr_crypt": (ctypes.c_int, [ctypes.POINTER(aes_sched_t), ctypes.c_char_p, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_void_p]),
    "aes_ctr_crypt_cfg": (ctypes.c_int, [ctypes.POINTER(aes_sched_t), ctypes.c_char_p,
                                         ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.POINTER(aes_launch_cfg_t),
                                         ctypes.c_void_p]),
    "aes_ctr_crypt_batch": (ctypes.c_int, [ctypes.POINTER(aes_ctr_desc_t), ctypes.c_size_t,
                                           ctypes.c_void_p]),
    "aes_ctr_crypt_batch_cfg": (ctypes.c_int, [ctypes.POINTER(aes_ctr_desc_t), ctypes.c_size_t,
                                               ctypes.POINTER(aes_batch_cfg_t), ctypes.c_void_p]),
    "aes_ctr_crypt_batch_noalloc": (ctypes.c_int, [ctypes.POINTER(aes_ctr_desc_t), ctypes.c_size_t,
                                                   ctypes.c_void_p]),
    "aes_engine_create": (ctypes.c_int, [ctypes.POINTER(aes_engine_cfg_t),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "aes_engine_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aes_ctr_desc_t),
                                  ctypes.POINTER(ctypes.c_uint64)]),
    "aes_submit_at": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aes_ctr_desc_t), ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_uint64)]),
    "aes_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "aes_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64]),
    "aes_engine_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(aes_stats_t)]),
    "aes_engine_reset_stats": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_engine_completion_fd": (ctypes.c_int, [ctypes.c_void_p]),
    "aes_engine_request_overhead": (ctypes.c_uint64, []),
    "aes_ctr_launch_shape": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(aes_launch_cfg_t),
                                            ctypes.POINTER(aes_launch_cfg_t)]),
    "sha256_batch": (ctypes.c_int, [ctypes.POINTER(sha256_desc_t), ctypes.c_size_t, ctypes.c_void_p]),
}


def _bind_torch_runtime() -> None:
    """One HIP runtime per process.  PyTorch ships its own libamdhip64 and
    libhsa-runtime64 (sonames libamdhip64.so.7 / libhsa-runtime64.so.1) but
    asks for them by another file name, so if this library loaded first, with
    ROCm's copies, PyTorch would load a second pair: two runtimes whose
    streams and devices do not mix.  Loading PyTorch first makes this
    library's dependencies resolve to PyTorch's already-loaded copies."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    _bind_torch_runtime()
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = load()
