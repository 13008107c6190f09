"""Host-side checks of libaesctr.so that need no GPU.

* the library loads and exports every function include/aesctr.h declares;
* aes_expand_key (host code of the product, written independently of the
  oracle) equals the oracle's FIPS-197 KeyExpansion;
* argument validation returns the documented status before any device work.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2607_02630_amd as A
from paper_2607_02630_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions() -> list[str]:
    """Every function declared by the library's headers (aesctr.h, shabatch.h)."""
    names = set()
    for hdr, prefix in (("aesctr.h", "aes_"), ("shabatch.h", "sha256_")):
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(" + prefix + r"\w+)\s*\(", text))
    return sorted(names)


def test_every_declared_function_is_exported():
    names = header_functions()
    assert len(names) >= 14
    L = ctypes.CDLL(N.LIB_PATH)
    for name in names:
        assert hasattr(L, name), f"{name} declared but not exported"
    assert set(names) == set(N.SIGNATURES), "binding and header disagree"


def test_strerror_names_every_status():
    for code in range(0, -12, -1):
        assert A.aes_strerror(code).startswith("AES_")
    assert "unknown" in A.aes_strerror(-99)


@pytest.mark.parametrize("klen", [16, 32])
def test_expand_key_matches_oracle(klen):
    g = np.random.default_rng(klen)
    for _ in range(200):
        key = g.bytes(klen)
        s = A.aes_expand_key(key)
        nr, w = oracle.expand(key)
        assert s.nr == nr and s.key_bits == 8 * klen
        assert list(s.rk[:4 * (nr + 1)]) == w


def test_expand_key_rejects_bad_sizes():
    for klen in (0, 15, 24, 31, 33):
        with pytest.raises(A.AesError) as e:
            A.aes_expand_key(bytes(klen))
        assert e.value.status == N.AES_EINVAL
    assert A.lib.aes_expand_key(None, 128, None) == N.AES_EINVAL


def _crypt_rc(sched, nonce, ctr0, src, dst, n):
    return A.lib.aes_ctr_crypt(ctypes.byref(sched) if sched is not None else None,
                               nonce, ctr0, src, dst, n, None)


def test_validation_before_device():
    s = A.aes_expand_key(bytes(16))
    nonce = bytes(12)
    # len == 0 is a no-op, even with null buffers.
    assert _crypt_rc(s, nonce, 1, None, None, 0) == N.AES_OK
    assert _crypt_rc(None, nonce, 1, 0x1000, 0x2000, 16) == N.AES_EINVAL
    assert _crypt_rc(s, None, 1, 0x1000, 0x2000, 16) == N.AES_EINVAL
    assert _crypt_rc(s, nonce, 1, None, 0x2000, 16) == N.AES_EINVAL
    assert _crypt_rc(s, nonce, 1, 0x1000, None, 16) == N.AES_EINVAL
    # Partial overlap (in place is fine, checked on the GPU).
    assert _crypt_rc(s, nonce, 1, 0x1000, 0x1008, 16) == N.AES_EOVERLAP
    assert _crypt_rc(s, nonce, 1, 0x1008, 0x1000, 16) == N.AES_EOVERLAP
    # More than 2^32 blocks.
    assert _crypt_rc(s, nonce, 1, 0x1000, 0x10000000000000, (1 << 36) + 16) == N.AES_ERANGE
    # A corrupted schedule.
    bad = A.aes_expand_key(bytes(16))
    bad.nr = 12
    assert _crypt_rc(bad, nonce, 1, 0x1000, 0x2000, 16) == N.AES_EINVAL
    bad = A.aes_expand_key(bytes(32))
    bad.key_bits = 128
    assert _crypt_rc(bad, nonce, 1, 0x1000, 0x2000, 16) == N.AES_EINVAL


def test_launch_cfg_validation():
    s = A.aes_expand_key(bytes(16))
    for kw in (dict(variant=4), dict(blocks_per_lane=3), dict(wg_size=100), dict(wg_size=2048),
               dict(grid=-1), dict(lds_copies=16), dict(lds_tables=3), dict(lds_copies=64, lds_tables=4),
               dict(wave_groups=4), dict(wave_groups=-1)):
        cfg = A.launch_cfg(**kw)
        rc = A.lib.aes_ctr_crypt_cfg(ctypes.byref(s), bytes(12), 1, 0x1000, 0x2000, 16,
                                     ctypes.byref(cfg), None)
        assert rc == N.AES_EINVAL, kw


def test_loadgen_library_exports_its_header():
    text = open(os.path.join(ROOT, "include", "aesloadgen.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(aes_load_\w+)\s*\(", text)))
    assert names == ["aes_load_engine", "aes_load_sync", "aes_load_sync_host"]
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2607_02630_amd", "libaesloadgen.so"))
    for name in names:
        assert hasattr(L, name)


def test_loadgen_validation_without_device():
    from paper_2607_02630_amd import loadgen
    res = loadgen.aes_load_result_t()
    assert loadgen.lib.aes_load_engine(None, None, 0, None, 0, ctypes.byref(res)) == N.AES_EINVAL
    assert loadgen.lib.aes_load_sync(None, 0, None, 0, None, ctypes.byref(res)) == N.AES_EINVAL
    assert loadgen.lib.aes_load_sync_host(None, 0, None, 0, None, 0, None, ctypes.byref(res)) == N.AES_EINVAL


def test_engine_entry_points_reject_null_handles():
    L = A.lib
    t = ctypes.c_uint64()
    assert L.aes_engine_create(None, None) == N.AES_EINVAL
    assert L.aes_engine_destroy(None) == N.AES_EINVAL
    assert L.aes_submit(None, None, ctypes.byref(t)) == N.AES_EINVAL
    assert L.aes_submit_at(None, None, 0, ctypes.byref(t)) == N.AES_EINVAL
    assert L.aes_poll(None, 1) == N.AES_EINVAL
    assert L.aes_wait(None, 1, 0) == N.AES_EINVAL
    assert L.aes_engine_stats(None, None) == N.AES_EINVAL
    assert L.aes_engine_reset_stats(None) == N.AES_EINVAL
    assert L.aes_engine_completion_fd(None) == N.AES_EINVAL
    # Without a GPU the engine cannot start.
    h = ctypes.c_void_p()
    assert L.aes_engine_create(None, ctypes.byref(h)) in (N.AES_EDEVICE, N.AES_OK)
    if h.value:
        L.aes_engine_destroy(h)


def test_sha_header_functions_are_exported_and_bound():
    text = open(os.path.join(ROOT, "include", "shabatch.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(sha256_\w+)\s*\(", text)))
    assert names == ["sha256_batch"]
    L = ctypes.CDLL(N.LIB_PATH)
    for name in names:
        assert hasattr(L, name)
        assert name in N.SIGNATURES


def test_sha_validation_before_device():
    arr = (N.sha256_desc_t * 2)()
    L = A.lib
    assert L.sha256_batch(None, 0, None) == N.AES_OK
    assert L.sha256_batch(None, 1, None) == N.AES_EINVAL
    arr[0].in_, arr[0].len, arr[0].digest = 0x1000, 16, None
    assert L.sha256_batch(arr, 1, None) == N.AES_EINVAL          # no digest buffer
    arr[0].digest = 0x1008
    assert L.sha256_batch(arr, 1, None) == N.AES_EOVERLAP        # digest inside its input
    arr[0].digest = 0x0ff0
    assert L.sha256_batch(arr, 1, None) == N.AES_EOVERLAP        # digest runs into its input
    arr[0].digest, arr[0].reserved = 0x9000, 1
    assert L.sha256_batch(arr, 1, None) == N.AES_EINVAL
    arr[0].reserved, arr[0].len = 0, 1 << 61
    assert L.sha256_batch(arr, 1, None) == N.AES_ERANGE          # bit length would overflow
    arr[0].len, arr[0].in_ = 5, None
    assert L.sha256_batch(arr, 1, None) == N.AES_EINVAL
    # The second descriptor is checked too.
    arr[0].in_ = 0x1000
    arr[1].in_, arr[1].len, arr[1].digest, arr[1].reserved = 0x2000, 8, 0x3000, 7
    assert L.sha256_batch(arr, 2, None) == N.AES_EINVAL


def test_sha_validation_of_a_large_batch_reports_the_first_error():
    # Large batches are validated in parallel parts (here four, of 17,500
    # descriptors); the status is still the one of the first failing
    # descriptor, as a serial scan would return.
    n = 70_000
    arr = (N.sha256_desc_t * n)()
    v = np.frombuffer(arr, dtype=np.uint64).reshape(n, 4)
    idx = np.arange(n, dtype=np.uint64)
    v[:, 0] = 0x10_0000_0000 + idx * 4096         # input
    v[:, 1] = 4096                                # length
    v[:, 2] = 0x20_0000_0000 + idx * 32           # digest
    v[:, 3] = 0                                   # reserved
    v[66_000, 3] = 1                              # EINVAL, last
    v[50_000, 1] = 1 << 61                        # ERANGE
    v[30_000, 2] = v[30_000, 0] + 64              # EOVERLAP, first
    assert A.lib.sha256_batch(arr, n, None) == N.AES_EOVERLAP
    v[30_000, 2] = 0x20_0000_0000 + 30_000 * 32
    assert A.lib.sha256_batch(arr, n, None) == N.AES_ERANGE
    v[50_000, 1] = 4096
    assert A.lib.sha256_batch(arr, n, None) == N.AES_EINVAL


def test_batch_validation_of_a_large_batch_reports_the_first_error():
    n = 10_000   # two parts of 5,000 descriptors
    s = A.aes_expand_key(bytes(16))
    bad = A.aes_expand_key(bytes(16))
    bad.nr = 12
    arr = (N.aes_ctr_desc_t * n)()
    for i in range(n):
        d = arr[i]
        d.in_ = 0x10_0000_0000 + i * 8192
        d.out = 0x20_0000_0000 + i * 8192
        d.len = 4096
        d.sched = ctypes.pointer(s)
    arr[9_000].flags = 3                          # EINVAL, last
    arr[7_000].len = (1 << 36) + 16               # ERANGE
    arr[3_000].out = arr[3_000].in_ + 8           # EOVERLAP, first
    assert A.lib.aes_ctr_crypt_batch(arr, n, None) == N.AES_EOVERLAP
    arr[3_000].out = 0x20_0000_0000 + 3_000 * 8192
    assert A.lib.aes_ctr_crypt_batch(arr, n, None) == N.AES_ERANGE
    arr[7_000].len = 4096
    arr[8_000].sched = ctypes.pointer(bad)        # EINVAL, before the flags one
    assert A.lib.aes_ctr_crypt_batch(arr, n, None) == N.AES_EINVAL


def test_binding_refuses_undersized_tensors_before_any_launch():
    """A tensor smaller than the bytes asked for is refused in Python, before
    the library is called, so no kernel can read or write past it (CPU
    tensors stand in for device ones: the check never reaches the device)."""
    import torch
    import paper_2607_02630_amd as A
    s = A.aes_expand_key(bytes(16))
    x64, x32 = torch.zeros(64, dtype=torch.uint8), torch.zeros(32, dtype=torch.uint8)
    with pytest.raises(ValueError, match="out holds 32 bytes"):
        A.aes_ctr_crypt(s, bytes(12), 0, x64, out=x32)
    with pytest.raises(ValueError, match="x holds 64 bytes"):
        A.aes_ctr_crypt(s, bytes(12), 0, x64, out=torch.zeros(128, dtype=torch.uint8), length=100)
    with pytest.raises(ValueError, match="length"):
        A.aes_ctr_crypt(s, bytes(12), 0, x64, out=x64, length=-1)
    with pytest.raises(ValueError, match="out holds 32 bytes"):
        A.Request(s, bytes(12), 0, x64, x32)
    with pytest.raises(ValueError, match="x holds 64 bytes"):
        A.Request(s, bytes(12), 0, x64, 0x1000, length=65)
    with pytest.raises(ValueError, match="digest holds 16 bytes"):
        A.HashRequest(x64, torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError, match="message 0 holds 64 bytes"):
        A.make_sha_desc_array([(x64, 65, torch.zeros(32, dtype=torch.uint8))])
    # Tensors that are large enough pass the check (raw addresses are the
    # caller's responsibility).
    A.Request(s, bytes(12), 0, x64, x64, length=64)
    A.HashRequest(x64, torch.zeros(32, dtype=torch.uint8))
