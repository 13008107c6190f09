"""GPU parity of aes_ctr_crypt_batch (one persistent launch over a table).

Every request is checked against the CPU oracle: fully for batches the
oracle finishes in seconds, by sampled blocks (first, last/partial, random
interior) for the 4096-request workload (log-uniform 4 KiB..8 MiB, mixed
AES-128/AES-256 keys, random nonces and start counters).  Also: edge cases
(empty requests, partial blocks, unaligned and in-place buffers, counter
wrap), more requests than one launch takes, order invariance, graph and
plain launch, and replays with new contents.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log, torch_cuda

pytestmark = pytest.mark.gpu


def lib():
    import paper_2607_02630_amd as A
    return A


class Batch:
    """Requests carved out of one input and one output device buffer."""

    def __init__(self, torch, reqs, in_place=False, misalign=False, seed=0):
        self.reqs = reqs
        offs, pos = [], 0
        for i, r in enumerate(reqs):
            pad = (i * 7) % 16 if misalign else 0
            pos += pad
            offs.append(pos)
            pos += r.length
            pos = (pos + 255) // 256 * 256 if not misalign else pos
        self.total = max(pos, 1)
        self.src = W.device_payload(self.total, seed)
        self.dst = self.src.clone() if in_place else torch.zeros_like(self.src)
        self.offs = offs
        self.in_place = in_place
        A = lib()
        self.scheds = [A.aes_expand_key(r.key) for r in reqs]
        base_in = self.dst.data_ptr() if in_place else self.src.data_ptr()
        self.objs = [A.Request(s, r.nonce, r.ctr0, base_in + o, self.dst.data_ptr() + o, r.length)
                     for s, r, o in zip(self.scheds, reqs, offs)]

    def run(self, cfg=None, order=None):
        A = lib()
        objs = self.objs if order is None else [self.objs[i] for i in order]
        A.aes_ctr_crypt_batch(objs, cfg=cfg)

    def host_in(self, i, a=0, b=None):
        r = self.reqs[i]
        b = r.length if b is None else b
        o = self.offs[i]
        return self.src[o + a:o + b].cpu().numpy()

    def host_out(self, i, a=0, b=None):
        r = self.reqs[i]
        b = r.length if b is None else b
        o = self.offs[i]
        return self.dst[o + a:o + b].cpu().numpy()

    def check_full(self, i):
        r = self.reqs[i]
        ref = oracle.ctr(r.key, r.nonce, r.ctr0, self.host_in(i), threads=0)
        assert np.array_equal(self.host_out(i), ref), f"request {i} len {r.length}"

    def check_sampled(self, i, rng):
        r = self.reqs[i]
        nb = (r.length + 15) // 16
        blocks = {0, nb - 1, int(rng.integers(0, nb))}
        for j in sorted(blocks):
            a, b = 16 * j, min(16 * j + 16, r.length)
            ref = oracle.ctr(r.key, r.nonce, (r.ctr0 + j) & 0xFFFFFFFF, self.host_in(i, a, b))
            assert np.array_equal(self.host_out(i, a, b), ref), f"request {i} block {j}"


def small_mix(n, seed, lo=1, hi=200_000):
    g = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        bits = 128 if i % 2 == 0 else 256
        length = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        reqs.append(W.Request(g.bytes(bits // 8), g.bytes(12), int(g.integers(0, 1 << 32)), length))
    return reqs


@pytest.mark.parametrize("use_graph", [1, 0])
def test_small_mixed_batch_full_parity(use_graph):
    torch = torch_cuda()
    reqs = small_mix(300, 11)
    reqs[5].length = 0
    reqs[17].ctr0 = 0xFFFFFFF0          # wraps inside the request
    reqs[30].length = 15
    b = Batch(torch, reqs, seed=5)
    b.run(cfg=lib().batch_cfg(use_graph=use_graph))
    torch.cuda.synchronize()
    for i in range(len(reqs)):
        if reqs[i].length:
            b.check_full(i)


@pytest.mark.parametrize("tile_bytes", [1024, 4096, 65536])
@pytest.mark.parametrize("bpl", [1, 2])
def test_tiling_shapes(tile_bytes, bpl):
    torch = torch_cuda()
    reqs = small_mix(64, 12, lo=1000, hi=300_000)
    b = Batch(torch, reqs, seed=6)
    b.run(cfg=lib().batch_cfg(tile_bytes=tile_bytes, blocks_per_lane=bpl, grid=37))
    torch.cuda.synchronize()
    for i in range(len(reqs)):
        b.check_full(i)


@pytest.mark.parametrize("n", [1, 2, 5, 8, 9])
@pytest.mark.parametrize("misalign", [False, True])
def test_small_batches_through_kernel_arguments(n, misalign):
    # Up to 8 requests travel in the kernel's argument block (no table
    # upload, static tile assignment); 9 takes the table path.  Lengths up to
    # 3 MB give several tiles per request; empty, 15-byte and wrapping
    # requests are mixed in.
    torch = torch_cuda()
    reqs = small_mix(n, 100 + n, lo=1, hi=3_000_000)
    if n >= 5:
        reqs[1].length = 0
        reqs[2].length = 15
        reqs[3].ctr0 = 0xFFFFFF00
    reqs[-1].length = 0 if n == 9 else reqs[-1].length
    b = Batch(torch, reqs, misalign=misalign, seed=n)
    for cfg in (None, lib().batch_cfg(tile_bytes=2048, grid=3)):
        b.dst.zero_()
        b.run(cfg=cfg)
        torch.cuda.synchronize()
        for i in range(n):
            if reqs[i].length:
                b.check_full(i)


def test_unaligned_and_in_place():
    torch = torch_cuda()
    reqs = small_mix(80, 13, lo=1, hi=50_000)
    b = Batch(torch, reqs, misalign=True, seed=7)
    b.run()
    torch.cuda.synchronize()
    for i in range(len(reqs)):
        b.check_full(i)
    b2 = Batch(torch, small_mix(40, 14, lo=16, hi=80_000), in_place=True, seed=8)
    plain = b2.src.clone()
    b2.run()
    torch.cuda.synchronize()
    for i, r in enumerate(b2.reqs):
        o = b2.offs[i]
        ref = oracle.ctr(r.key, r.nonce, r.ctr0, plain[o:o + r.length].cpu().numpy())
        assert np.array_equal(b2.dst[o:o + r.length].cpu().numpy(), ref)


def test_more_requests_than_one_launch_and_order_invariance():
    torch = torch_cuda()
    reqs = small_mix(4096 + 700, 15, lo=16, hi=4096)
    b = Batch(torch, reqs, seed=9)
    b.run()
    torch.cuda.synchronize()
    first = b.dst.clone()
    rng = np.random.default_rng(1)
    for i in rng.choice(len(reqs), 200, replace=False):
        b.check_full(int(i))
    b.dst.zero_()
    b.run(order=list(rng.permutation(len(reqs))))
    torch.cuda.synchronize()
    assert torch.equal(first, b.dst)


def test_replays_with_new_contents():
    """Consecutive calls reuse staging slots and graphs; each must use its
    own descriptors."""
    torch = torch_cuda()
    batches = [Batch(torch, small_mix(50, 20 + k, lo=16, hi=100_000), seed=30 + k) for k in range(6)]
    for bt in batches:
        bt.run()
    torch.cuda.synchronize()
    for bt in batches:
        for i in range(0, len(bt.reqs), 5):
            bt.check_full(i)


def test_batch_of_4096_loguniform_workload():
    """The full-size batch workload: every request sampled against the
    oracle, and equal to its own single-request call."""
    torch = torch_cuda()
    A = lib()
    reqs = W.batch_requests()
    log(f"batch: {len(reqs)} requests, {sum(r.length for r in reqs) / 2**30:.2f} GiB")
    b = Batch(torch, reqs, seed=4242)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for i in range(len(reqs)):
        b.check_sampled(i, rng)
    # Alone: each request through the single-buffer call into a fresh buffer.
    alone = torch.zeros_like(b.dst)
    for s, r, o in zip(b.scheds, reqs, b.offs):
        A.aes_ctr_crypt(s, r.nonce, r.ctr0, b.src.data_ptr() + o, alone.data_ptr() + o, length=r.length)
    torch.cuda.synchronize()
    assert torch.equal(alone, b.dst)


def test_batch_rejects_bad_requests():
    torch = torch_cuda()
    A = lib()
    import ctypes
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    s = A.aes_expand_key(bytes(16))
    good = A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr(), 64)
    bad = A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr() + 8, 64)
    arr = A.make_desc_array([good, bad])
    assert A.lib.aes_ctr_crypt_batch(arr, 2, torch.cuda.current_stream().cuda_stream) == -8
    d = good.desc()
    d.flags = 1
    arr = (A.aes_ctr_desc_t * 1)(d)
    assert A.lib.aes_ctr_crypt_batch(arr, 1, torch.cuda.current_stream().cuda_stream) == -1
    assert A.lib.aes_ctr_crypt_batch(None, 0, None) == 0
    assert A.lib.aes_ctr_crypt_batch(ctypes.cast(None, ctypes.POINTER(A.aes_ctr_desc_t)), 3, None) == -1
