"""Batched SHA-256 on the GPU against the SHA-256 oracle (FIPS 180-4).

Every digest is compared byte for byte with oracle/sharef.c (itself pinned
to hashlib and to the constants' definitions in test_oracle_sha.py).
Cases: every length 0..300 in one launch (all padding boundaries), mixed
large lengths, unaligned inputs and digests, more messages than one launch
holds, and the benchmark's workload at full size (sampled).
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import sha
from gpu_util import log, torch_cuda

pytestmark = pytest.mark.gpu


def lib():
    import paper_2607_02630_amd as A
    return A


def gpu_hash(msgs: list[bytes], in_align: int = 0, dig_align: int = 0, pad: int = 0) -> list[bytes]:
    """Hash host messages on the GPU: packed into one device buffer (each
    message starting at an offset congruent to in_align mod 16), digests at
    offsets congruent to dig_align."""
    torch = torch_cuda()
    A = lib()
    offs, o = [], 0
    for m in msgs:
        o = (o + 15) // 16 * 16 + in_align
        offs.append(o)
        o += len(m) + pad
    buf = np.zeros(max(o, 1), dtype=np.uint8)
    for m, off in zip(msgs, offs):
        buf[off:off + len(m)] = np.frombuffer(m, dtype=np.uint8)
    dev = torch.from_numpy(buf).cuda()
    dig = torch.zeros(48 * len(msgs) + 16, dtype=torch.uint8, device="cuda")
    base_in, base_d = dev.data_ptr(), dig.data_ptr()
    items = [(base_in + off, len(m), base_d + 48 * i + dig_align) for i, (m, off) in enumerate(zip(msgs, offs))]
    A.sha256_batch(items)
    torch.cuda.synchronize()
    h = dig.cpu().numpy()
    return [h[48 * i + dig_align:48 * i + dig_align + 32].tobytes() for i in range(len(msgs))]


def test_every_length_0_to_300_in_one_launch():
    g = np.random.default_rng(1)
    msgs = [g.bytes(n) for n in range(301)]
    log("sha256 lengths 0..300")
    got = gpu_hash(msgs)
    for n, (m, d) in enumerate(zip(msgs, got)):
        assert d == sha.sha256(m), n


def test_mixed_large_lengths():
    g = np.random.default_rng(2)
    lens = [4096, 65536, 1 << 20, 1000003, 64, 0, 4095, 123457, 8 << 20]
    msgs = [g.bytes(n) for n in lens]
    log("sha256 mixed large")
    got = gpu_hash(msgs)
    for m, d in zip(msgs, got):
        assert d == sha.sha256(m), len(m)


@pytest.mark.parametrize("in_align,dig_align", [(1, 0), (3, 5), (8, 12), (0, 7)])
def test_unaligned_inputs_and_digests(in_align, dig_align):
    g = np.random.default_rng(in_align * 16 + dig_align)
    msgs = [g.bytes(int(n)) for n in g.integers(0, 3000, size=97)]
    log(f"sha256 unaligned {in_align} {dig_align}")
    got = gpu_hash(msgs, in_align=in_align, dig_align=dig_align)
    for m, d in zip(msgs, got):
        assert d == sha.sha256(m), len(m)


def test_more_messages_than_one_launch():
    """267,144 messages exceed one launch's table (131,072): the call splits
    into three launches."""
    g = np.random.default_rng(3)
    n = (1 << 18) + 5000
    lens = g.integers(0, 200, size=n)
    msgs = [g.bytes(int(k)) for k in lens]
    log(f"sha256 {n} messages")
    got = gpu_hash(msgs)
    for i in range(n):
        assert got[i] == sha.sha256(msgs[i]), i


def test_benchmark_workload_sampled():
    """262,144 messages of 4 KiB (1 GiB) from the benchmark's generator;
    1,000 sampled digests checked against the oracle."""
    torch = torch_cuda()
    A = lib()
    import workloads as W
    n, size = W.HASH_MESSAGES, W.HASH_MESSAGE_BYTES
    log("sha256 1 GiB workload")
    src = W.device_payload(n * size, W.seed_for(7))
    dig = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
    items = [(src.data_ptr() + i * size, size, dig.data_ptr() + 32 * i) for i in range(n)]
    A.sha256_batch(items)
    torch.cuda.synchronize()
    idx = np.random.default_rng(4).choice(n, size=1000, replace=False)
    host = src.view(n, size)[torch.from_numpy(idx).cuda()].cpu().numpy()
    d = dig.view(n, 32).cpu().numpy()
    for k, i in enumerate(idx):
        assert d[i].tobytes() == sha.sha256(host[k].tobytes()), int(i)


@pytest.mark.parametrize("busy", [False, True], ids=["idle-stream", "busy-stream"])
def test_records_in_place_and_uploaded(busy):
    """A launch on an idle stream reads its records from pinned staging over
    PCIe; on a busy stream (here behind a 256 MiB AES launch) they are
    uploaded on a side stream first.  Two calls in a row, so the second
    reuses the staging the first filled."""
    torch = torch_cuda()
    A = lib()
    g = np.random.default_rng(21 if busy else 22)
    n = 3000
    msgs = [g.bytes(int(k)) for k in g.integers(0, 3000, size=n)]
    offs = np.cumsum([0] + [len(m) for m in msgs])
    buf = torch.from_numpy(np.frombuffer(b"".join(msgs) or b"\0", dtype=np.uint8).copy()).cuda()
    big = torch.zeros(256 << 20, dtype=torch.uint8, device="cuda")
    s = A.aes_expand_key(bytes(16))
    for rep in range(2):
        dig = torch.zeros(32 * n, dtype=torch.uint8, device="cuda")
        items = [(buf.data_ptr() + int(offs[i]), len(m), dig.data_ptr() + 32 * i) for i, m in enumerate(msgs)]
        torch.cuda.synchronize()
        if busy:
            A.aes_ctr_crypt(s, bytes(12), 1, big, big)      # keeps the stream busy for ~0.2 ms
        A.sha256_batch(items)
        torch.cuda.synchronize()
        h = dig.cpu().numpy()
        for i in range(n):
            assert h[32 * i:32 * i + 32].tobytes() == sha.sha256(msgs[i]), (rep, i)
