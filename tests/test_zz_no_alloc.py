"""aes_ctr_crypt_batch_noalloc (no allocation; its table in a fixed device
array of the library) against aes_ctr_crypt_batch, bit for bit, on two calls
in a row, the second with fewer and smaller requests (so stale table
contents from the first call would show), and against the oracle on sampled
blocks.  Called through the C ABI."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log, torch_cuda

pytestmark = pytest.mark.gpu


def make(torch, n, seed, lo, hi):
    import paper_2607_02630_amd as A
    g = np.random.default_rng(seed)
    lens = [int(x) for x in np.floor(np.exp(g.uniform(np.log(lo), np.log(hi), size=n)))]
    offs, pos = [], 0
    for L in lens:
        pos += int(g.integers(0, 16))        # some unaligned starts
        offs.append(pos)
        pos += L
    src = W.device_payload(pos + 64, seed)
    a = torch.zeros_like(src)
    b = torch.zeros_like(src)
    keys = [g.bytes(16 if i % 2 else 32) for i in range(n)]
    meta = [(k, g.bytes(12), int(g.integers(0, 1 << 32))) for k in keys]
    scheds = [A.aes_expand_key(k) for k in keys]
    ra = [A.Request(s, nonce, c, src.data_ptr() + o, a.data_ptr() + o, L)
          for s, (_, nonce, c), o, L in zip(scheds, meta, offs, lens)]
    rb = [A.Request(s, nonce, c, src.data_ptr() + o, b.data_ptr() + o, L)
          for s, (_, nonce, c), o, L in zip(scheds, meta, offs, lens)]
    torch.cuda.synchronize()
    return src, a, b, ra, rb, meta, offs, lens


def check(torch, A, n, seed, lo, hi):
    src, a, b, ra, rb, meta, offs, lens = make(torch, n, seed, lo, hi)
    log(f"no-alloc batch: {n} requests, {sum(lens)} bytes")
    da = A.make_desc_array(ra)
    st = torch.cuda.current_stream().cuda_stream
    assert A.lib.aes_ctr_crypt_batch_noalloc(da, n, st) == 0
    A.aes_ctr_crypt_batch(rb)
    torch.cuda.synchronize()
    assert torch.equal(a, b), "no-alloc output differs from aes_ctr_crypt_batch"
    rng = np.random.default_rng(seed + 1)
    for i in rng.choice(n, min(n, 24), replace=False):
        key, nonce, c = meta[i]
        nb = (lens[i] + 15) // 16
        for j in (0, nb - 1):
            s, e = offs[i] + 16 * j, min(offs[i] + 16 * j + 16, offs[i] + lens[i])
            ref = oracle.ctr(key, nonce, (c + j) & 0xFFFFFFFF, src[s:e].cpu().numpy())
            assert np.array_equal(a[s:e].cpu().numpy(), ref), (i, j)


def test_no_alloc_batch_equals_batch_twice():
    torch = torch_cuda()
    import paper_2607_02630_amd as A
    check(torch, A, 300, 901, 4096, 1 << 19)     # first call: 300 requests up to 512 KiB
    check(torch, A, 13, 902, 17, 70000)          # second call, smaller: 13 requests, odd lengths


def test_no_alloc_batch_limits():
    torch = torch_cuda()
    import paper_2607_02630_amd as A
    from paper_2607_02630_amd import _native as N
    st = torch.cuda.current_stream().cuda_stream
    arr = (N.aes_ctr_desc_t * 1)()
    assert A.lib.aes_ctr_crypt_batch_noalloc(arr, 4097, st) == N.AES_ETOOBIG
    assert A.lib.aes_ctr_crypt_batch_noalloc(None, 3, st) == N.AES_EINVAL
    assert A.lib.aes_ctr_crypt_batch_noalloc(None, 0, st) == N.AES_OK
