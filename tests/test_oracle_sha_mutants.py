"""The SHA-256 oracle's pins catch plausible mistakes (no GPU).

Each case copies oracle/sharef.c into a temporary directory, plants one
mistake by text substitution (a wrong rotation, a dropped term, a swapped
function, a wrong constant derivation, a padding or byte-order slip), builds
it with gcc and checks that the hashlib comparison rejects the mutant.  The
committed oracle is never modified.
"""
from __future__ import annotations

import contextlib
import hashlib
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sha

SRC = os.path.join(os.path.dirname(sha.__file__), "sharef.c")
HDR = os.path.join(os.path.dirname(sha.__file__), "sharef.h")

MUTANTS = {
    "big_sigma0_rotation": ("rotr(x, 2) ^ rotr(x, 13) ^ rotr(x, 22)", "rotr(x, 2) ^ rotr(x, 13) ^ rotr(x, 21)"),
    "small_sigma0_rotate_not_shift": ("rotr(x, 18) ^ (x >> 3)", "rotr(x, 18) ^ rotr(x, 3)"),
    "small_sigma1_dropped_term": ("rotr(x, 17) ^ rotr(x, 19) ^ (x >> 10)", "rotr(x, 17) ^ (x >> 10)"),
    "ch_operands_swapped": ("(x & y) ^ (~x & z)", "(x & z) ^ (~x & y)"),
    "maj_as_xor3": ("(x & y) ^ (x & z) ^ (y & z)", "x ^ y ^ z"),
    "schedule_index": ("W[t - 7] + small_sigma0(W[t - 15])", "W[t - 6] + small_sigma0(W[t - 15])"),
    "k_from_square_roots": ("k[i] = frac_root_bits(p[i], 3);", "k[i] = frac_root_bits(p[i], 2);"),
    "h0_from_cube_roots": ("h[i] = frac_root_bits(p[i], 2);", "h[i] = frac_root_bits(p[i], 3);"),
    "length_in_bytes": ("const uint64_t bits = len * 8;", "const uint64_t bits = len;"),
    "padding_boundary": ("rest + 1 + 8 <= 64", "rest + 8 <= 64"),
    "message_word_little_endian": ("W[t] = (uint32_t)block[4 * t] << 24", "W[t] = (uint32_t)block[4 * t + 3] << 24"),
    "feed_forward_dropped": ("    H[7] += h;\n", "\n"),
    "t2_without_maj": ("const uint32_t T2 = big_sigma0(a) + maj(a, b, c);", "const uint32_t T2 = big_sigma0(a);"),
}


@contextlib.contextmanager
def mutant_oracle(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    d = tmp_path / name
    d.mkdir()
    (d / "sharef.c").write_text(src.replace(old, new, 1))
    shutil.copy(HDR, d / "sharef.h")
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", str(so), str(d / "sharef.c")], check=True)
    saved = sha._lib
    sha._lib = sha.load_from(str(so))
    try:
        yield
    finally:
        sha._lib = saved


def pins_pass() -> bool:
    g = np.random.default_rng(5)
    for n in (0, 3, 55, 56, 63, 64, 65, 119, 120, 200):
        m = g.bytes(n)
        if sha.sha256(m) != hashlib.sha256(m).digest():
            return False
    return True


def test_unmutated_oracle_passes():
    assert pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    with mutant_oracle(tmp_path, name):
        assert not pins_pass(), f"mutant {name} slipped through"
