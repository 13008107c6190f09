"""The oracle's pins catch plausible mistakes (no GPU).

Each case copies the oracle source into a temporary directory, plants one
mistake by text substitution (a dropped term, a wrong direction or index, a
transposed operand, a wrong constant or byte order), builds it with gcc, and
checks that the pin checks reject the mutant.  The committed oracle is never
modified.
"""
from __future__ import annotations

import contextlib
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import _openssl
from test_oracle import independent_sbox

SRC = os.path.join(os.path.dirname(oracle.__file__), "aesref.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "aesref.h")

MUTANTS = {
    "shiftrows_wrong_direction": ("row[c] = s[r][(c + r) % 4];", "row[c] = s[r][(c - r + 4) % 4];"),
    "mixcolumns_transposed_coefficients": ("{0x02, 0x03, 0x01, 0x01}", "{0x02, 0x01, 0x03, 0x01}"),
    "mixcolumns_index_sign": ("coef[(k - r + 4) % 4]", "coef[(r - k + 4) % 4]"),
    "affine_constant": ("const uint8_t c = 0x63;", "const uint8_t c = 0x62;"),
    "affine_dropped_term": ("bit_of(b, i + 6) ^\n                bit_of(b, i + 7)",
                            "bit_of(b, i + 6)"),
    "rcon_off_by_one": ("aesref_rcon(i / nk)", "aesref_rcon(i / nk + 1)"),
    "aes256_extra_subword_dropped": ("nk > 6 && i % nk == 4", "nk > 8 && i % nk == 4"),
    "roundkey_byte_order": ("(uint8_t)(word >> (24 - 8 * r))", "(uint8_t)(word >> (8 * r))"),
    "counter_little_endian": ("out[12] = (uint8_t)(ctr >> 24);", "out[15] = (uint8_t)(ctr >> 24);"),
    "last_round_keeps_mixcolumns": ("    sub_bytes(s);\n    shift_rows(s);\n    add_round_key(s, w, nr);",
                                    "    sub_bytes(s);\n    shift_rows(s);\n    mix_columns(s);\n"
                                    "    add_round_key(s, w, nr);"),
    "partial_block_uses_suffix": ("out[off + b] = in[off + b] ^ o[b];",
                                  "out[off + b] = in[off + b] ^ o[16 - n + b];"),
    "counter_carry_into_nonce": ("    memcpy(out, nonce, 12);\n    out[12]",
                                 "    memcpy(out, nonce, 12);\n"
                                 "    if (((uint64_t)ctr0 + j) >> 32) out[11] += 1;\n    out[12]"),
    "xtime_wrong_reduction": ("shifted ^ 0x1b", "shifted ^ 0x1d"),
}


@contextlib.contextmanager
def mutant_oracle(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    d = tmp_path / name
    d.mkdir()
    (d / "aesref.c").write_text(src.replace(old, new, 1))
    shutil.copy(HDR, d / "aesref.h")
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-pthread", "-o", str(so),
                    str(d / "aesref.c")], check=True)
    saved = oracle._lib
    oracle._lib = oracle.load_from(str(so))
    try:
        yield
    finally:
        oracle._lib = saved


def pins_pass() -> bool:
    """A compact run of the pins in test_oracle.py against the loaded build."""
    if list(oracle.sbox()) != independent_sbox():
        return False
    for i in range(1, 11):
        if oracle.rcon(i + 1) != oracle.gf_mul(oracle.rcon(i), 2):
            return False
    g = np.random.default_rng(3)
    for klen in (16, 32):
        for _ in range(8):
            key, block = g.bytes(klen), g.bytes(16)
            if oracle.encrypt_block(key, block) != _openssl.ecb_encrypt_block(key, block):
                return False
            if oracle.decrypt_block(key, oracle.encrypt_block(key, block)) != block:
                return False
        nonce = g.bytes(12)
        for ctr0, n in ((1, 40), (0xFFFFFFFF, 37), (0xFFFFFFF0, 16 * 20 + 3)):
            data = g.bytes(n)
            if bytes(oracle.ctr(key, nonce, ctr0, data)) != _openssl.ctr_inc32(key, nonce, ctr0, data):
                return False
    return True


@pytest.mark.skipif(not _openssl.available(), reason="libcrypto not found")
def test_unmodified_oracle_passes_compact_pins():
    assert pins_pass()


@pytest.mark.skipif(not _openssl.available(), reason="libcrypto not found")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    with mutant_oracle(tmp_path, name):
        assert not pins_pass(), f"mutant {name} slipped through the pins"
