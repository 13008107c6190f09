"""GPU tests of the serving engine (submit -> poll/wait, continuous batching).

Each result is the same alone and in the mix (tolerance 0 bits): requests of
the serving size mix run through the engine concurrently, from several
submitting threads, and every output equals the single-request call on the
same input and the CPU oracle on sampled blocks.  Also: the byte budget
holds, oversize requests are refused, ticket semantics, pinned host buffers,
shutdown drains submitted work, and the completion file descriptor.
"""
from __future__ import annotations

import os
import select
import threading

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log, torch_cuda

pytestmark = pytest.mark.gpu

KiB, MiB = 1024, 1 << 20


def lib():
    import paper_2607_02630_amd as A
    return A


def make_requests(torch, n, seed, sizes=W.SERVING_SIZES, mix=W.SERVING_MIX, host=False):
    g = np.random.default_rng(seed)
    which = g.choice(len(sizes), size=n, p=mix)
    lens = [int(sizes[k]) for k in which]
    total = sum(lens)
    src = W.device_payload(total, seed)
    if host:
        src = src.cpu().pin_memory()
        dst = torch.zeros(total, dtype=torch.uint8).pin_memory()
    else:
        dst = torch.zeros_like(src)
    A = lib()
    reqs, offs, pos = [], [], 0
    for L in lens:
        key, nonce, ctr0 = g.bytes(16), g.bytes(12), int(g.integers(0, 1 << 32))
        s = A.aes_expand_key(key)
        reqs.append((key, nonce, ctr0, s, A.Request(s, nonce, ctr0, src.data_ptr() + pos, dst.data_ptr() + pos, L)))
        offs.append(pos)
        pos += L
    torch.cuda.synchronize()        # the engine's streams are not ordered after torch's
    return src, dst, reqs, offs, lens


def check_alone_and_oracle(torch, src, dst, reqs, offs, lens, rng):
    A = lib()
    dsrc = src.cuda() if not src.is_cuda else src
    alone = torch.zeros(dsrc.numel(), dtype=torch.uint8, device="cuda")
    for (key, nonce, ctr0, s, _), o, L in zip(reqs, offs, lens):
        A.aes_ctr_crypt(s, nonce, ctr0, dsrc.data_ptr() + o, alone.data_ptr() + o, length=L)
    torch.cuda.synchronize()
    got = dst.cuda() if not dst.is_cuda else dst
    assert torch.equal(alone, got), "engine output differs from the single-request call"
    for i in rng.choice(len(reqs), min(40, len(reqs)), replace=False):
        key, nonce, ctr0, _, _ = reqs[i]
        o, L = offs[i], lens[i]
        nb = L // 16
        for j in (0, nb - 1, int(rng.integers(0, nb))):
            a, b = o + 16 * j, o + 16 * j + 16
            ref = oracle.ctr(key, nonce, (ctr0 + j) & 0xFFFFFFFF, src[a:b].cpu().numpy())
            assert np.array_equal(got[a:b].cpu().numpy(), ref)


def test_same_alone_and_in_the_mix():
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_requests(torch, 600, 1)
    log(f"engine: {len(reqs)} requests, {sum(lens) / MiB:.1f} MiB")
    with A.Engine(budget_bytes=4 << 30, n_streams=2) as eng:
        tickets = [None] * len(reqs)

        def submit_range(lo, hi):
            for i in range(lo, hi):
                tickets[i] = eng.submit(reqs[i][4])

        ths = [threading.Thread(target=submit_range, args=(k * 150, (k + 1) * 150)) for k in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        for t in tickets:
            eng.wait(t)
        st = eng.stats()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["batches"] >= 1 and st["p99_us"] >= st["p50_us"] > 0
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(3))


def test_budget_is_respected():
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_requests(torch, 120, 2, sizes=(1 * MiB, 8 * MiB), mix=(0.6, 0.4))
    # An out-of-place 8 MiB request holds 16 MiB of buffers plus its record.
    budget = 24 * MiB
    with A.Engine(budget_bytes=budget, n_streams=2) as eng:
        ts = [eng.submit(r[4]) for r in reqs]
        for t in ts:
            eng.wait(t)
        st = eng.stats()
    assert 0 < st["budget_high_water"] <= budget
    assert st["batches"] >= 2 * sum(lens) // budget
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(4))


def test_oversize_and_ticket_semantics():
    torch = torch_cuda()
    A = lib()
    buf = torch.zeros(4 * MiB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = A.aes_expand_key(bytes(16))
    with A.Engine(budget_bytes=1 * MiB) as eng:
        with pytest.raises(A.AesError) as e:
            eng.submit(A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr(), 2 * MiB))
        assert e.value.status == -3
        with pytest.raises(A.AesError) as e:
            eng.submit(A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr() + 8, 64))
        assert e.value.status == -8
        t = eng.submit(A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr(), 512 * KiB))
        eng.wait(t)
        with pytest.raises(A.AesError) as e:
            eng.poll(t)                      # retired by wait
        assert e.value.status == -6
        with pytest.raises(A.AesError):
            eng.wait(123456789, 1000)
        t2 = eng.submit(A.Request(s, bytes(12), 1, buf.data_ptr(), buf.data_ptr(), 0))
        eng.wait(t2, 5_000_000)
        st = eng.stats()
        assert st["rejected"] == 1


def test_pinned_host_buffers():
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_requests(torch, 60, 5, sizes=(64 * KiB, 1 * MiB), mix=(0.7, 0.3),
                                               host=True)
    with A.Engine(budget_bytes=256 * MiB, host_buffers=True) as eng:
        ts = [eng.submit(r[4]) for r in reqs]
        for t in ts:
            eng.wait(t)
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(6))


def test_pinned_host_buffers_large_requests_alone():
    # Each request runs as a batch of its own, so a zero-copy launch takes
    # its larger tiles (several steps per wave); odd lengths leave the later
    # requests unaligned and with partial final blocks.
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_requests(torch, 8, 9, sizes=(8 * MiB + 5, 3 * MiB + 17, 64 * KiB + 1),
                                               mix=(0.4, 0.3, 0.3), host=True)
    log(f"pinned alone: {[L for L in lens]}")
    with A.Engine(budget_bytes=256 * MiB, host_buffers=True) as eng:
        for r in reqs:
            eng.wait(eng.submit(r[4]))
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(10))


def test_destroy_drains_submitted_work():
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_requests(torch, 200, 7)
    eng = A.Engine()
    for r in reqs:
        eng.submit(r[4])
    eng.close()                 # returns after every submitted request ran
    torch.cuda.synchronize()
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(8))


def test_completion_fd_becomes_readable():
    torch = torch_cuda()
    A = lib()
    buf = torch.zeros(MiB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = A.aes_expand_key(bytes(32))
    with A.Engine() as eng:
        fd = eng.completion_fd()
        t = eng.submit(A.Request(s, bytes(12), 7, buf.data_ptr(), buf.data_ptr(), MiB))
        r, _, _ = select.select([fd], [], [], 10.0)
        assert fd in r
        os.read(fd, 8)
        assert eng.poll(t) or (eng.wait(t) is None)


def test_mixed_cipher_and_hash_requests():
    """Cipher and SHA-256 requests through one engine: every ciphertext
    equals the oracle's AES-CTR and every digest the SHA-256 oracle's, with
    launches that carry both kinds.  Hash requests include the empty
    message, unaligned inputs and a digest at an odd address."""
    from oracle import sha
    torch = torch_cuda()
    A = lib()
    g = np.random.default_rng(77)
    n = 400
    kinds = g.integers(0, 2, size=n)                  # 0 cipher, 1 hash
    lens = [int(x) for x in g.integers(0, 200_000, size=n)]
    lens[3], lens[5] = 0, 1
    total = sum(lens) + 16 * n
    src_h = np.frombuffer(g.bytes(total), dtype=np.uint8).copy()
    src = torch.from_numpy(src_h).cuda()
    dst = torch.zeros(total, dtype=torch.uint8, device="cuda")
    dig = torch.zeros(33 * n + 1, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    reqs, meta, pos = [], [], 0
    for i in range(n):
        pos += int(g.integers(0, 16))                  # unaligned starts
        L = lens[i]
        if kinds[i] == 0 and L > 0:
            key, nonce, ctr0 = g.bytes(16), g.bytes(12), int(g.integers(0, 1 << 32))
            reqs.append(A.Request(A.aes_expand_key(key), nonce, ctr0, src.data_ptr() + pos, dst.data_ptr() + pos, L))
            meta.append(("aes", pos, L, key, nonce, ctr0))
        else:
            reqs.append(A.HashRequest(src.data_ptr() + pos, dig.data_ptr() + 33 * i + 1, L))
            meta.append(("sha", pos, L, i))
        pos += L
    log("engine mixed cipher + hash")
    with A.Engine(budget_bytes=64 * MiB) as eng:
        tickets = [eng.submit(r) for r in reqs]
        for t in tickets:
            eng.wait(t)
        assert eng.stats()["batches"] >= 1
    out = dst.cpu().numpy()
    dg = dig.cpu().numpy()
    for m in meta:
        if m[0] == "aes":
            _, p, L, key, nonce, ctr0 = m
            assert np.array_equal(out[p:p + L], oracle.ctr(key, nonce, ctr0, src_h[p:p + L])), p
        else:
            _, p, L, i = m
            assert dg[33 * i + 1:33 * i + 33].tobytes() == sha.sha256(src_h[p:p + L].tobytes()), i


def test_hash_request_validation():
    torch = torch_cuda()
    A = lib()
    from paper_2607_02630_amd import _native as N
    import ctypes
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with A.Engine(budget_bytes=16 * MiB) as eng:
        t = ctypes.c_uint64()
        d = A.HashRequest(buf, buf.data_ptr() + 16, 64).desc()      # digest inside the message
        assert A.lib.aes_submit(eng._h, ctypes.byref(d), ctypes.byref(t)) == N.AES_EOVERLAP
        d = A.HashRequest(buf, None, 64).desc()
        assert A.lib.aes_submit(eng._h, ctypes.byref(d), ctypes.byref(t)) == N.AES_EINVAL
        d = A.HashRequest(buf, buf.data_ptr() + 2048, 64).desc()
        d.reserved = 1
        assert A.lib.aes_submit(eng._h, ctypes.byref(d), ctypes.byref(t)) == N.AES_EINVAL
        d.flags = 2                                                    # unknown flag
        d.reserved = 0
        assert A.lib.aes_submit(eng._h, ctypes.byref(d), ctypes.byref(t)) == N.AES_EINVAL


def make_tenant_requests(torch, n, n_keys, seed, sizes=(4 * KiB, 64 * KiB, 1 * MiB + 7), mix=(0.5, 0.4, 0.1)):
    """Requests whose keys repeat: each draws one of n_keys tenant keys (half
    AES-128, half AES-256), with its own nonce and start counter."""
    g = np.random.default_rng(seed)
    keys = [g.bytes(16 if i % 2 == 0 else 32) for i in range(n_keys)]
    scheds = [lib().aes_expand_key(k) for k in keys]
    which = g.choice(len(sizes), size=n, p=mix)
    lens = [int(sizes[k]) for k in which]
    src = W.device_payload(sum(lens), seed)
    dst = torch.zeros_like(src)
    A = lib()
    reqs, offs, pos = [], [], 0
    for L in lens:
        k = int(g.integers(0, n_keys))
        nonce, ctr0 = g.bytes(12), int(g.integers(0, 1 << 32))
        reqs.append((keys[k], nonce, ctr0, scheds[k],
                     A.Request(scheds[k], nonce, ctr0, src.data_ptr() + pos, dst.data_ptr() + pos, L)))
        offs.append(pos)
        pos += L
    torch.cuda.synchronize()
    return src, dst, reqs, offs, lens


@pytest.mark.parametrize("n_keys,slots", [(6, 16), (40, 16)], ids=["fits", "evicts"])
def test_resident_key_slots(n_keys, slots):
    """Key schedules resident in the engine's key slots.  Requests reuse a few
    tenant keys: first one at a time (single-request launches, whose
    records travel in the kernel arguments, install and then hit slots),
    then in bursts (launches through the staged table).  With more keys than
    slots the least recently used ones are evicted and re-installed.  Every
    output equals the single-request call and the oracle, and every cipher
    request counts as a hit or a miss."""
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_tenant_requests(torch, 500, n_keys, 31 + n_keys)
    log(f"key slots: {n_keys} keys, {slots} slots, {len(reqs)} requests")
    with A.Engine(key_slots=slots, n_streams=2) as eng:
        for r in reqs[:60]:
            eng.wait(eng.submit(r[4]))
        st1 = eng.stats()
        for lo in range(60, len(reqs), 110):
            ts = [eng.submit(r[4]) for r in reqs[lo:lo + 110]]
            for t in ts:
                eng.wait(t)
        st = eng.stats()
    assert st["key_hits"] + st["key_misses"] == len(reqs)
    if n_keys <= slots:
        # One at a time, each key misses once (its install), then hits.
        assert st1["key_hits"] >= 60 - 2 * n_keys
        assert st["key_hits"] > len(reqs) * 3 // 4
    else:
        # Uniform draws over more keys than slots: about slots / keys hit.
        assert st["key_hits"] > len(reqs) // 8
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(n_keys))


def test_without_key_slots_nothing_is_counted():
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_tenant_requests(torch, 50, 3, 5)
    with A.Engine() as eng:
        for t in [eng.submit(r[4]) for r in reqs]:
            eng.wait(t)
        st = eng.stats()
    assert st["key_hits"] == 0 and st["key_misses"] == 0
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(5))


@pytest.mark.parametrize("in_place", [False, True], ids=["out_of_place", "in_place"])
def test_budget_counts_device_bytes(in_place):
    """The admission weight of a cipher request is its buffers (input and
    output, once when in place) plus its staged records; with one request in
    flight the budget's high-water mark is exactly that."""
    torch = torch_cuda()
    A = lib()
    n = 8 * MiB
    buf = torch.zeros(2 * n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    s = A.aes_expand_key(bytes(range(16)))
    out = buf.data_ptr() if in_place else buf.data_ptr() + n
    overhead = A.lib.aes_engine_request_overhead()
    assert overhead == 64 + 256
    with A.Engine() as eng:
        eng.wait(eng.submit(A.Request(s, bytes(12), 1, buf.data_ptr(), out, n)))
        st = eng.stats()
    assert st["budget_high_water"] == (1 if in_place else 2) * n + overhead
    got = buf[n:].cpu().numpy() if not in_place else buf[:n].cpu().numpy()
    ref = oracle.ctr(bytes(range(16)), bytes(12), 1, np.zeros(n, np.uint8))
    assert np.array_equal(got[:4096], ref[:4096]) and np.array_equal(got[-4096:], ref[-4096:])


def test_engines_do_not_grow_device_memory():
    """Creating and destroying engines reuses the staging of retired
    streams: 64 engines, each running a batch through the staged table (more
    than 8 requests), a hash request and key slots, leave device memory
    where it was (within a few MiB)."""
    torch = torch_cuda()
    A = lib()
    src, dst, reqs, offs, lens = make_tenant_requests(torch, 24, 4, 71, sizes=(64 * KiB,), mix=(1.0,))
    dig = torch.zeros(32, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def one_engine():
        with A.Engine(key_slots=8, n_streams=2) as eng:
            ts = [eng.submit(r[4]) for r in reqs]
            ts.append(eng.submit(A.HashRequest(src, dig, 4096)))
            for t in ts:
                eng.wait(t)

    for _ in range(4):          # the pools reach their steady size
        one_engine()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for i in range(64):
        one_engine()
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log(f"free device memory {free0 / MiB:.1f} -> {free1 / MiB:.1f} MiB after 64 engines")
    assert free0 - free1 < 4 * MiB
    check_alone_and_oracle(torch, src, dst, reqs, offs, lens, np.random.default_rng(72))
