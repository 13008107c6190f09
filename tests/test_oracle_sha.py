"""Pins of the SHA-256 oracle (no GPU).

The oracle (oracle/sharef.c, FIPS 180-4) is checked against things other
than itself:
* Python's hashlib (OpenSSL's SHA-256, a library routine) on every length
  from 0 to 300 bytes, which crosses each padding boundary (55/56 bytes: the
  length field still fits / spills into a second block; 63/64/65; 119/120)
  and on larger messages;
* the properties the constants' definitions fix, checked with Python's
  exact integers by a different method (Newton iteration on the integer
  root, not the oracle's bisection): each K_t is the floor of the cube root
  of p * 2^96 mod 2^32, each H0 word the floor of the square root of
  p * 2^64 mod 2^32, over the first 64 / 8 primes found by trial division;
* invariants: messages differing in one bit or one length give different
  digests; the multithreaded driver equals the single-message call.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np
import pytest

from oracle import sha


def _is_prime(n: int) -> bool:
    return n >= 2 and all(n % d for d in range(2, int(math.isqrt(n)) + 1))


def _iroot_newton(x: int, e: int) -> int:
    """floor(x ** (1/e)) by integer Newton iteration."""
    if x < 2:
        return x
    y = 1 << ((x.bit_length() + e - 1) // e)
    while True:
        z = ((e - 1) * y + x // y ** (e - 1)) // e
        if z >= y:
            break
        y = z
    while y ** e > x:
        y -= 1
    while (y + 1) ** e <= x:
        y += 1
    return y


def test_primes():
    p = sha.primes(64)
    assert p == [n for n in range(2, 312) if _is_prime(n)]


def test_constants_from_their_definitions():
    p = [n for n in range(2, 312) if _is_prime(n)]
    k = [_iroot_newton(q << 96, 3) % (1 << 32) for q in p]
    h = [_iroot_newton(q << 64, 2) % (1 << 32) for q in p[:8]]
    assert sha.k_constants() == k
    assert sha.h0() == h


@pytest.mark.parametrize("lo,hi", [(0, 100), (100, 200), (200, 301)])
def test_every_short_length_matches_hashlib(lo, hi):
    g = np.random.default_rng(lo)
    for n in range(lo, hi):
        m = g.bytes(n)
        assert sha.sha256(m) == hashlib.sha256(m).digest(), n


@pytest.mark.parametrize("n", [1000, 4095, 4096, 4097, 65536, (1 << 20) + 7])
def test_long_messages_match_hashlib(n):
    m = np.random.default_rng(n).bytes(n)
    assert sha.sha256(m) == hashlib.sha256(m).digest()


def test_structured_inputs():
    for m in (b"", b"\x00" * 64, b"\xff" * 56, bytes(range(256)) * 3, b"\x80" + b"\x00" * 62):
        assert sha.sha256(m) == hashlib.sha256(m).digest()


def test_avalanche_and_length():
    g = np.random.default_rng(9)
    m = bytearray(g.bytes(200))
    d0 = sha.sha256(bytes(m))
    m[77] ^= 0x10
    assert sha.sha256(bytes(m)) != d0
    assert sha.sha256(bytes(m[:199])) != sha.sha256(bytes(m))


@pytest.mark.parametrize("threads", [1, 3])
def test_many_equals_single(threads):
    g = np.random.default_rng(threads)
    msgs = np.frombuffer(g.bytes(37 * 129), dtype=np.uint8).reshape(37, 129)
    out, used = sha.sha256_many(msgs, threads)
    assert used == threads
    for i in range(37):
        assert bytes(out[i]) == hashlib.sha256(msgs[i].tobytes()).digest()
