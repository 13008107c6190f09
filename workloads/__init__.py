"""Seeded synthetic inputs for the AES-CTR and batched SHA-256 workloads.

This module only draws random bytes and sizes; it holds none of the cipher's
arithmetic, so both the GPU path's tests and the CPU oracle can consume the
same host bytes.  Generator: numpy ``Generator(PCG64(seed))``.

Workloads (payloads are uniform random bytes; sizes in binary KiB/MiB):

* ``single``   one 1 MiB buffer, AES-128, ctr0 = 1.
* ``sweep``    AES-128 or AES-256, powers of two 4 KiB .. 8 MiB plus 256 MiB,
               ctr0 = 1.
* ``batch``    4096 requests, lengths log-uniform on [4 KiB, 8 MiB] in exact
               bytes (floor(exp(U(ln 4096, ln 8388608)))), exactly half
               AES-128 and half AES-256 keys in shuffled order, random nonce
               and random 32-bit start counter per request.
* ``serving``  open-loop Poisson arrivals (exponential gaps) with sizes
               70% 64 KiB / 25% 1 MiB / 5% 8 MiB, AES-128 key, nonce and
               start counter per request.
* ``hash``     262,144 messages of 4 KiB (1 GiB) of uniform random bytes,
               generated on the GPU with seed 2607 * 10 + 7.

Seeds: master 2607, workload k uses 2607 * 10 + k (k = 1..5, 7).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASTER_SEED = 2607
KiB = 1024
MiB = 1024 * 1024
SWEEP_SIZES = [4 * KiB << i for i in range(12)]      # 4 KiB .. 8 MiB
BIG_SIZE = 256 * MiB
# Batched hashing: many independent messages of one size (1 GiB in all).
HASH_MESSAGES = 262144
HASH_MESSAGE_BYTES = 4 * KiB


def seed_for(k: int) -> int:
    return MASTER_SEED * 10 + k


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def payload(g: np.random.Generator, nbytes: int) -> np.ndarray:
    return np.frombuffer(g.bytes(nbytes), dtype=np.uint8).copy()


@dataclass
class Stream:
    """One message: key, nonce, start counter and payload bytes."""
    key: bytes
    nonce: bytes
    ctr0: int
    data: np.ndarray


def single_1mib() -> Stream:
    g = rng(seed_for(1))
    key = g.bytes(16)
    nonce = g.bytes(12)
    return Stream(key, nonce, 1, payload(g, 1 * MiB))


def sweep_key(key_bits: int) -> tuple[bytes, bytes]:
    """Key and nonce of the single-buffer sweep (AES-128: k=2, AES-256: k=3)."""
    g = rng(seed_for(2 if key_bits == 128 else 3))
    return g.bytes(key_bits // 8), g.bytes(12)


def sweep_payload(nbytes: int, key_bits: int) -> np.ndarray:
    g = rng(seed_for(2 if key_bits == 128 else 3) * 1000 + int(math.log2(nbytes)))
    return payload(g, nbytes)


@dataclass
class Request:
    key: bytes
    nonce: bytes
    ctr0: int
    length: int


def batch_requests(n: int = 4096, lo: int = 4 * KiB, hi: int = 8 * MiB,
                   seed: int | None = None) -> list[Request]:
    g = rng(seed_for(4) if seed is None else seed)
    u = g.uniform(math.log(lo), math.log(hi), size=n)
    lengths = np.floor(np.exp(u)).astype(np.int64)
    lengths = np.clip(lengths, lo, hi)
    bits = np.array([128] * (n // 2) + [256] * (n - n // 2))
    g.shuffle(bits)
    reqs = []
    for i in range(n):
        key = g.bytes(int(bits[i]) // 8)
        nonce = g.bytes(12)
        ctr0 = int(g.integers(0, 1 << 32))
        reqs.append(Request(key, nonce, ctr0, int(lengths[i])))
    return reqs


SERVING_SIZES = (64 * KiB, 1 * MiB, 8 * MiB)
SERVING_MIX = (0.70, 0.25, 0.05)


def serving_trace(n: int, rate_per_s: float, seed: int | None = None):
    """Arrival times (seconds, from 0), sizes and per-request key material."""
    g = rng(seed_for(5) if seed is None else seed)
    gaps = g.exponential(1.0 / rate_per_s, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = g.choice(3, size=n, p=SERVING_MIX)
    sizes = np.array(SERVING_SIZES, dtype=np.int64)[which]
    keys = [g.bytes(16) for _ in range(n)]
    nonces = [g.bytes(12) for _ in range(n)]
    ctr0s = g.integers(0, 1 << 32, size=n, dtype=np.uint64)
    return arrivals, sizes, keys, nonces, ctr0s


def device_payload(nbytes: int, seed: int):
    """Uniform random bytes generated on the GPU (torch's seeded generator),
    for batches too large to stage from the host; the same bytes can be
    copied back for the oracle."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    chunk = 1 << 28
    for a in range(0, nbytes, chunk):
        b = min(nbytes, a + chunk)
        out[a:b] = torch.randint(0, 256, (b - a,), dtype=torch.uint8, device="cuda", generator=g)
    return out
