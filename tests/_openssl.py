"""OpenSSL's libcrypto, run as a library: an independent AES to pin the oracle.

Only the EVP interface is used (``EVP_aes_*_ecb`` for single blocks,
``EVP_aes_*_ctr`` for counter mode).  OpenSSL's CTR increments the whole
128-bit counter block, carrying into the nonce, whereas the reading used here
wraps only the low 32 bits (inc32, NIST SP 800-38A Appendix B).  ``ctr_inc32``
therefore splits a message at every 2^32 wrap of the counter and restarts
OpenSSL at ``nonce || 00000000`` for each piece.
"""
from __future__ import annotations

import ctypes
import ctypes.util

_crypto = None


def available() -> bool:
    try:
        _load()
        return True
    except OSError:
        return False


def _load():
    global _crypto
    if _crypto is not None:
        return _crypto
    name = ctypes.util.find_library("crypto") or "libcrypto.so.3"
    L = ctypes.CDLL(name)
    L.EVP_CIPHER_CTX_new.restype = ctypes.c_void_p
    L.EVP_CIPHER_CTX_free.argtypes = [ctypes.c_void_p]
    for fn in ("EVP_aes_128_ecb", "EVP_aes_192_ecb", "EVP_aes_256_ecb",
               "EVP_aes_128_ctr", "EVP_aes_192_ctr", "EVP_aes_256_ctr"):
        getattr(L, fn).restype = ctypes.c_void_p
    L.EVP_EncryptInit_ex.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_char_p, ctypes.c_char_p]
    L.EVP_EncryptInit_ex.restype = ctypes.c_int
    L.EVP_DecryptInit_ex.argtypes = L.EVP_EncryptInit_ex.argtypes
    L.EVP_DecryptInit_ex.restype = ctypes.c_int
    L.EVP_CIPHER_CTX_set_padding.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.EVP_EncryptUpdate.argtypes = [ctypes.c_void_p, ctypes.c_char_p,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_char_p, ctypes.c_int]
    L.EVP_EncryptUpdate.restype = ctypes.c_int
    L.EVP_DecryptUpdate.argtypes = L.EVP_EncryptUpdate.argtypes
    L.EVP_DecryptUpdate.restype = ctypes.c_int
    _crypto = L
    return L


def _cipher(mode: str, key_len: int):
    L = _load()
    return getattr(L, f"EVP_aes_{8 * key_len}_{mode}")()


def _run(mode: str, key: bytes, iv: bytes | None, data: bytes, decrypt: bool = False) -> bytes:
    L = _load()
    ctx = L.EVP_CIPHER_CTX_new()
    if not ctx:
        raise MemoryError("EVP_CIPHER_CTX_new")
    try:
        init = L.EVP_DecryptInit_ex if decrypt else L.EVP_EncryptInit_ex
        upd = L.EVP_DecryptUpdate if decrypt else L.EVP_EncryptUpdate
        if init(ctx, _cipher(mode, len(key)), None, key, iv) != 1:
            raise RuntimeError("EVP init failed")
        L.EVP_CIPHER_CTX_set_padding(ctx, 0)
        out = ctypes.create_string_buffer(len(data) + 32)
        outl = ctypes.c_int(0)
        done = 0
        chunk = 1 << 30
        res = bytearray()
        while done < len(data):
            piece = data[done:done + chunk]
            if upd(ctx, out, ctypes.byref(outl), piece, len(piece)) != 1:
                raise RuntimeError("EVP update failed")
            res += out.raw[:outl.value]
            done += len(piece)
        return bytes(res)
    finally:
        L.EVP_CIPHER_CTX_free(ctx)


def ecb_encrypt_block(key: bytes, block: bytes) -> bytes:
    assert len(block) == 16
    return _run("ecb", key, None, bytes(block))


def ecb_decrypt_block(key: bytes, block: bytes) -> bytes:
    assert len(block) == 16
    return _run("ecb", key, None, bytes(block), decrypt=True)


def ctr_inc32(key: bytes, nonce: bytes, ctr0: int, data: bytes) -> bytes:
    """CTR with a 32-bit big-endian counter that wraps without carrying."""
    out = bytearray()
    pos = 0
    ctr = ctr0 & 0xFFFFFFFF
    while pos < len(data) or (pos == 0 and not data):
        if not data:
            break
        blocks_to_wrap = (1 << 32) - ctr
        take = min(len(data) - pos, blocks_to_wrap * 16)
        iv = bytes(nonce) + ctr.to_bytes(4, "big")
        out += _run("ctr", key, iv, bytes(data[pos:pos + take]))
        pos += take
        ctr = 0
    return bytes(out)
