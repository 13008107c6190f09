"""CPU oracle for SHA-256 -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``liboracle_sharef.so``, plain C written from FIPS 180-4
(logical functions Sec. 4.1.2; constants Sec. 4.2.2 and the initial hash
value of Sec. 5.3.3, computed from their definitions; padding Sec. 5.1.1;
hash computation Sec. 6.2.2).  Only ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's ``cpu_baseline`` leg may import this module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_sharef.so")
_lib = None
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def load_from(path: str) -> ctypes.CDLL:
    L = ctypes.CDLL(path)
    L.sharef_primes.argtypes = [ctypes.c_int, _u32p]
    L.sharef_k.argtypes = [_u32p]
    L.sharef_h0.argtypes = [_u32p]
    L.sharef_sha256.argtypes = [ctypes.c_void_p, ctypes.c_uint64, _u8p]
    L.sharef_sha256_many.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_int]
    L.sharef_sha256_many.restype = ctypes.c_int
    return L


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            subprocess.run(["make", "-s", "-C", _HERE], check=True)
        _lib = load_from(_LIB_PATH)
    return _lib


def primes(n: int) -> list[int]:
    out = (ctypes.c_uint32 * n)()
    lib().sharef_primes(n, out)
    return list(out)


def k_constants() -> list[int]:
    out = (ctypes.c_uint32 * 64)()
    lib().sharef_k(out)
    return list(out)


def h0() -> list[int]:
    out = (ctypes.c_uint32 * 8)()
    lib().sharef_h0(out)
    return list(out)


def sha256(data) -> bytes:
    if isinstance(data, (bytes, bytearray, memoryview)):
        a = np.frombuffer(bytes(data), dtype=np.uint8)
    else:
        a = np.ascontiguousarray(data, dtype=np.uint8).reshape(-1)
    out = (ctypes.c_uint8 * 32)()
    lib().sharef_sha256(a.ctypes.data if a.size else None, a.size, out)
    return bytes(out)


def sha256_many(msgs: np.ndarray, threads: int = 1) -> tuple[np.ndarray, int]:
    """Digests of the rows of a 2-D uint8 array (equal-length messages);
    returns (digests [n, 32], threads used)."""
    m = np.ascontiguousarray(msgs, dtype=np.uint8)
    n, length = m.shape
    out = np.empty((n, 32), dtype=np.uint8)
    used = lib().sharef_sha256_many(m.ctypes.data if m.size else None, length, n, out.ctypes.data, threads)
    return out, used
