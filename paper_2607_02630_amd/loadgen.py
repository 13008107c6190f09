"""ctypes binding of libaesloadgen.so (include/aesloadgen.h): replay an
open-loop arrival schedule against the engine or the synchronous path."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _native as N

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaesloadgen.so")


class aes_load_result_t(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("achieved_rps", ctypes.c_double),
                ("gbps", ctypes.c_double), ("max_lag_us", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("p999_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("completed", ctypes.c_uint64), ("errors", ctypes.c_uint64)]


def _load():
    if not os.path.exists(_LIB):
        raise ImportError(f"{_LIB} is missing: build the library first")
    L = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    L.aes_load_engine.argtypes = [ctypes.c_void_p, ctypes.POINTER(N.aes_ctr_desc_t), ctypes.c_size_t,
                                  dp, ctypes.c_size_t, ctypes.POINTER(aes_load_result_t)]
    L.aes_load_engine.restype = ctypes.c_int
    L.aes_load_sync.argtypes = [ctypes.POINTER(N.aes_ctr_desc_t), ctypes.c_size_t, dp, ctypes.c_size_t,
                                ctypes.c_void_p, ctypes.POINTER(aes_load_result_t)]
    L.aes_load_sync.restype = ctypes.c_int
    L.aes_load_sync_host.argtypes = [ctypes.POINTER(N.aes_ctr_desc_t), ctypes.c_size_t, dp, ctypes.c_size_t,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.POINTER(aes_load_result_t)]
    L.aes_load_sync_host.restype = ctypes.c_int
    return L


lib = _load()


def _as_dict(r: aes_load_result_t) -> dict:
    return {name: getattr(r, name) for name, _ in aes_load_result_t._fields_}


def run_engine(engine, pool, arrivals_s: np.ndarray) -> dict:
    a = np.ascontiguousarray(arrivals_s, dtype=np.float64)
    res = aes_load_result_t()
    rc = lib.aes_load_engine(engine._h, pool, len(pool), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             a.size, ctypes.byref(res))
    if rc < 0:
        raise RuntimeError(N.lib.aes_strerror(rc).decode())
    return _as_dict(res)


def run_sync(pool, arrivals_s: np.ndarray, stream: int) -> dict:
    a = np.ascontiguousarray(arrivals_s, dtype=np.float64)
    res = aes_load_result_t()
    rc = lib.aes_load_sync(pool, len(pool), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size,
                           stream, ctypes.byref(res))
    if rc < 0:
        raise RuntimeError(N.lib.aes_strerror(rc).decode())
    return _as_dict(res)


def run_sync_host(pool, arrivals_s: np.ndarray, dev_buf: int, dev_bytes: int, stream: int) -> dict:
    """Synchronous per-request path for pinned-host payloads: copy in,
    encrypt on the device, copy out, synchronise, one request at a time."""
    a = np.ascontiguousarray(arrivals_s, dtype=np.float64)
    res = aes_load_result_t()
    rc = lib.aes_load_sync_host(pool, len(pool), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size,
                                dev_buf, dev_bytes, stream, ctypes.byref(res))
    if rc < 0:
        raise RuntimeError(N.lib.aes_strerror(rc).decode())
    return _as_dict(res)
