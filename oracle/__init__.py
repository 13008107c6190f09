"""CPU oracle for AES-CTR -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``liboracle_aesref.so``, the plain byte-oriented AES written
from the FIPS-197 definitions (field arithmetic Sec. 4, S-box Sec. 5.1.1,
round transformations Sec. 5.1, KeyExpansion Sec. 5.2, InvCipher Sec. 5.3)
with NIST SP 800-38A counter mode (Sec. 6.5, inc32 of Appendix B).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this module.  The product library shares no
code with it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_aesref.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build() -> str:
    """Compile the oracle with the Makefile beside it (gcc, -mno-aes)."""
    subprocess.run(["make", "-s", "-C", _HERE], check=True)
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """The oracle library, built on first use if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load_from(_LIB_PATH)
    return _lib


def load_from(path: str) -> ctypes.CDLL:
    """Load an oracle build from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    L.aesref_xtime.argtypes = [ctypes.c_uint8]
    L.aesref_xtime.restype = ctypes.c_uint8
    L.aesref_gf_mul.argtypes = [ctypes.c_uint8, ctypes.c_uint8]
    L.aesref_gf_mul.restype = ctypes.c_uint8
    L.aesref_gf_inv.argtypes = [ctypes.c_uint8]
    L.aesref_gf_inv.restype = ctypes.c_uint8
    L.aesref_sbox.argtypes = [_u8p]
    L.aesref_inv_sbox.argtypes = [_u8p]
    L.aesref_rcon.argtypes = [ctypes.c_int]
    L.aesref_rcon.restype = ctypes.c_uint8
    L.aesref_mix_column.argtypes = [_u8p]
    L.aesref_inv_mix_column.argtypes = [_u8p]
    L.aesref_expand.argtypes = [_u8p, ctypes.c_int, _u32p]
    L.aesref_expand.restype = ctypes.c_int
    L.aesref_encrypt_block.argtypes = [_u32p, ctypes.c_int, _u8p, _u8p]
    L.aesref_decrypt_block.argtypes = [_u32p, ctypes.c_int, _u8p, _u8p]
    L.aesref_counter_block.argtypes = [_u8p, ctypes.c_uint32, ctypes.c_uint64, _u8p]
    L.aesref_ctr.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_uint32,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64]
    L.aesref_ctr.restype = ctypes.c_int
    L.aesref_ctr_mt.argtypes = [_u8p, ctypes.c_int, _u8p, ctypes.c_uint32,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.c_int]
    L.aesref_ctr_mt.restype = ctypes.c_int
    return L


def _bytes_ptr(b: bytes):
    buf = (ctypes.c_uint8 * len(b)).from_buffer_copy(b)
    return buf, ctypes.cast(buf, _u8p)


def xtime(b: int) -> int:
    return lib().aesref_xtime(b)


def gf_mul(a: int, b: int) -> int:
    return lib().aesref_gf_mul(a, b)


def gf_inv(a: int) -> int:
    return lib().aesref_gf_inv(a)


def sbox() -> np.ndarray:
    out = (ctypes.c_uint8 * 256)()
    lib().aesref_sbox(out)
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


def inv_sbox() -> np.ndarray:
    out = (ctypes.c_uint8 * 256)()
    lib().aesref_inv_sbox(out)
    return np.frombuffer(bytes(out), dtype=np.uint8).copy()


def rcon(i: int) -> int:
    return lib().aesref_rcon(i)


def mix_column(col: bytes) -> bytes:
    buf = (ctypes.c_uint8 * 4).from_buffer_copy(bytes(col))
    lib().aesref_mix_column(buf)
    return bytes(buf)


def inv_mix_column(col: bytes) -> bytes:
    buf = (ctypes.c_uint8 * 4).from_buffer_copy(bytes(col))
    lib().aesref_inv_mix_column(buf)
    return bytes(buf)


def expand(key: bytes) -> tuple[int, list[int]]:
    """FIPS-197 KeyExpansion -> (Nr, [w_0 .. w_{4Nr+3}]) as big-endian words."""
    w = (ctypes.c_uint32 * 60)()
    _, kp = _bytes_ptr(key)
    nr = lib().aesref_expand(kp, 8 * len(key), w)
    if nr < 0:
        raise ValueError("key must be 16, 24 or 32 bytes")
    return nr, [int(w[i]) for i in range(4 * (nr + 1))]


def encrypt_block(key: bytes, block: bytes) -> bytes:
    nr, wl = expand(key)
    w = (ctypes.c_uint32 * 60)(*wl)
    src = (ctypes.c_uint8 * 16).from_buffer_copy(bytes(block))
    dst = (ctypes.c_uint8 * 16)()
    lib().aesref_encrypt_block(w, nr, src, dst)
    return bytes(dst)


def decrypt_block(key: bytes, block: bytes) -> bytes:
    nr, wl = expand(key)
    w = (ctypes.c_uint32 * 60)(*wl)
    src = (ctypes.c_uint8 * 16).from_buffer_copy(bytes(block))
    dst = (ctypes.c_uint8 * 16)()
    lib().aesref_decrypt_block(w, nr, src, dst)
    return bytes(dst)


def counter_block(nonce: bytes, ctr0: int, j: int) -> bytes:
    _, npp = _bytes_ptr(nonce)
    dst = (ctypes.c_uint8 * 16)()
    lib().aesref_counter_block(npp, ctr0 & 0xFFFFFFFF, j, dst)
    return bytes(dst)


def _as_u8(data) -> np.ndarray:
    if isinstance(data, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(data), dtype=np.uint8)
    a = np.ascontiguousarray(data)
    if a.dtype != np.uint8:
        raise TypeError("payload must be uint8")
    return a.reshape(-1)


def ctr(key: bytes, nonce: bytes, ctr0: int, data, threads: int = 1) -> np.ndarray:
    """AES-CTR of ``data`` (bytes or uint8 array) -> new uint8 array.

    ``threads`` > 1 (or 0 = all CPUs) uses the multithreaded driver, which
    splits the block range into contiguous per-thread pieces."""
    if len(key) not in (16, 24, 32) or len(nonce) != 12:
        raise ValueError("bad key or nonce length")
    src = _as_u8(data)
    dst = np.empty_like(src)
    _kb, kp = _bytes_ptr(key)
    _nb, npp = _bytes_ptr(nonce)
    n = src.size
    sp = src.ctypes.data if n else None
    dp = dst.ctypes.data if n else None
    if threads == 1:
        rc = lib().aesref_ctr(kp, 8 * len(key), npp, ctr0 & 0xFFFFFFFF, sp, dp, n)
    else:
        rc = lib().aesref_ctr_mt(kp, 8 * len(key), npp, ctr0 & 0xFFFFFFFF, sp, dp, n, threads)
    if rc < 0:
        raise ValueError("oracle rejected the arguments")
    return dst


def ctr_mt_timed(key: bytes, nonce: bytes, ctr0: int, src: np.ndarray, dst: np.ndarray,
                 threads: int) -> int:
    """Multithreaded CTR into a caller buffer; returns the threads used."""
    _kb, kp = _bytes_ptr(key)
    _nb, npp = _bytes_ptr(nonce)
    rc = lib().aesref_ctr_mt(kp, 8 * len(key), npp, ctr0 & 0xFFFFFFFF,
                             src.ctypes.data, dst.ctypes.data, src.size, threads)
    if rc < 0:
        raise ValueError("oracle rejected the arguments")
    return rc
