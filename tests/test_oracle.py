"""Pins for the CPU oracle (no GPU).

Each check ties the oracle to something other than itself: closed forms of
GF(2^8) arithmetic computed here by a different algorithm (carry-less product
then polynomial long division), exhaustive invariants of the S-box and of
MixColumns (FIPS-197 Sec. 4, 5.1.1, 5.1.3, 5.3), counter-mode identities
(NIST SP 800-38A Sec. 6.5 and Appendix B), and an independent AES -- OpenSSL's
libcrypto run as a library -- for KeyExpansion + Cipher (Sec. 5.1, 5.2) and
for counter mode split at 32-bit counter wraps.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import _openssl

M_X = 0x11B    # x^8 + x^4 + x^3 + x + 1


def clmul_mod(a: int, b: int) -> int:
    """Polynomial product over GF(2) followed by long division by m(x)."""
    p = 0
    for i in range(8):
        if (b >> i) & 1:
            p ^= a << i
    for deg in range(14, 7, -1):
        if (p >> deg) & 1:
            p ^= M_X << (deg - 8)
    return p


def rotl8(b: int, n: int) -> int:
    return ((b << n) | (b >> (8 - n))) & 0xFF


# --------------------------------------------------------------------------
# GF(2^8), FIPS-197 Sec. 4
# --------------------------------------------------------------------------

def test_xtime_closed_form():
    assert oracle.xtime(0x80) == 0x1B          # x^8 = x^4 + x^3 + x + 1 mod m(x)
    assert oracle.xtime(0x01) == 0x02
    for b in range(256):
        assert oracle.xtime(b) == clmul_mod(b, 2)


def test_gf_mul_exhaustive_against_long_division():
    for a in range(256):
        for b in range(256):
            assert oracle.gf_mul(a, b) == clmul_mod(a, b), (a, b)


def test_gf_inverse_exhaustive():
    assert oracle.gf_inv(0) == 0
    for a in range(1, 256):
        assert clmul_mod(a, oracle.gf_inv(a)) == 1, a


# --------------------------------------------------------------------------
# S-box, Sec. 5.1.1
# --------------------------------------------------------------------------

def independent_sbox() -> list[int]:
    """Inverse by exhaustive search; affine map in its rotation form
    b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ {63}."""
    inv = [0] * 256
    for a in range(1, 256):
        for b in range(1, 256):
            if clmul_mod(a, b) == 1:
                inv[a] = b
                break
    out = []
    for x in range(256):
        b = inv[x]
        out.append(b ^ rotl8(b, 1) ^ rotl8(b, 2) ^ rotl8(b, 3) ^ rotl8(b, 4) ^ 0x63)
    return out


def test_sbox_matches_independent_construction():
    assert list(oracle.sbox()) == independent_sbox()


def test_sbox_design_properties():
    s = oracle.sbox()
    assert s[0] == 0x63                          # 0^-1 := 0, then the affine constant
    assert sorted(s.tolist()) == list(range(256))  # bijection
    for x in range(256):
        assert s[x] != x                          # no fixed point
        assert s[x] != (x ^ 0xFF)                 # no "opposite" fixed point


def test_inverse_sbox_is_inverse_permutation():
    s, si = oracle.sbox(), oracle.inv_sbox()
    for x in range(256):
        assert si[s[x]] == x
        assert s[si[x]] == x


def test_rcon_powers_of_x():
    assert oracle.rcon(1) == 1
    for i in range(1, 15):
        assert oracle.rcon(i + 1) == clmul_mod(oracle.rcon(i), 2)
    assert oracle.rcon(9) == 0x1B and oracle.rcon(10) == 0x36  # x^8, x^9 reduced


# --------------------------------------------------------------------------
# MixColumns, Sec. 5.1.3 / 5.3.3
# --------------------------------------------------------------------------

def poly_mod_x4_plus_1(a_coef, b_coef):
    """(sum a_i x^i)(sum b_j x^j) mod x^4 + 1 over GF(2^8): x^4 = 1."""
    out = [0, 0, 0, 0]
    for i in range(4):
        for j in range(4):
            out[(i + j) % 4] ^= clmul_mod(a_coef[i], b_coef[j])
    return out


def test_mix_column_is_polynomial_product():
    a = [0x02, 0x01, 0x01, 0x03]          # a(x) = {03}x^3 + {01}x^2 + {01}x + {02}
    ainv = [0x0E, 0x09, 0x0D, 0x0B]      # a^-1(x) = {0b}x^3 + {0d}x^2 + {09}x + {0e}
    g = np.random.default_rng(11)
    for _ in range(300):
        col = list(g.integers(0, 256, size=4))
        col = [int(c) for c in col]
        assert list(oracle.mix_column(bytes(col))) == poly_mod_x4_plus_1(a, col)
        assert list(oracle.inv_mix_column(bytes(col))) == poly_mod_x4_plus_1(ainv, col)


def test_mix_columns_inverse_identity():
    assert poly_mod_x4_plus_1([0x02, 0x01, 0x01, 0x03], [0x0E, 0x09, 0x0D, 0x0B]) == [1, 0, 0, 0]
    g = np.random.default_rng(12)
    for _ in range(300):
        col = bytes(g.integers(0, 256, size=4, dtype=np.uint8))
        assert oracle.inv_mix_column(oracle.mix_column(col)) == col
        assert oracle.mix_column(oracle.inv_mix_column(col)) == col


# --------------------------------------------------------------------------
# KeyExpansion + Cipher, Sec. 5.1 / 5.2 / 5.3
# --------------------------------------------------------------------------

@pytest.mark.parametrize("klen,nr", [(16, 10), (24, 12), (32, 14)])
def test_key_expansion_shape(klen, nr):
    g = np.random.default_rng(klen)
    key = g.bytes(klen)
    got_nr, w = oracle.expand(key)
    assert got_nr == nr and len(w) == 4 * (nr + 1)
    nk = klen // 4
    for i in range(nk):
        assert w[i] == int.from_bytes(key[4 * i:4 * i + 4], "big")


def test_key_expansion_recurrence_rederived():
    """w[i] = w[i-Nk] ^ temp with the rules of Sec. 5.2, recomputed here on top
    of the independently built S-box."""
    s = independent_sbox()

    def sub_word(x):
        return int.from_bytes(bytes(s[b] for b in x.to_bytes(4, "big")), "big")

    g = np.random.default_rng(5)
    for klen in (16, 24, 32):
        key = g.bytes(klen)
        nr, w = oracle.expand(key)
        nk = klen // 4
        rc = 1
        for i in range(nk, 4 * (nr + 1)):
            t = w[i - 1]
            if i % nk == 0:
                t = sub_word(((t << 8) | (t >> 24)) & 0xFFFFFFFF) ^ (rc << 24)
                rc = clmul_mod(rc, 2)
            elif nk > 6 and i % nk == 4:
                t = sub_word(t)
            assert w[i] == w[i - nk] ^ t, (klen, i)


needs_openssl = pytest.mark.skipif(not _openssl.available(), reason="libcrypto not found")


@needs_openssl
@pytest.mark.parametrize("klen", [16, 24, 32])
def test_cipher_matches_openssl(klen):
    g = np.random.default_rng(100 + klen)
    for _ in range(200):
        key, block = g.bytes(klen), g.bytes(16)
        assert oracle.encrypt_block(key, block) == _openssl.ecb_encrypt_block(key, block)
        assert oracle.decrypt_block(key, block) == _openssl.ecb_decrypt_block(key, block)


@pytest.mark.parametrize("klen", [16, 24, 32])
def test_decrypt_inverts_encrypt(klen):
    g = np.random.default_rng(200 + klen)
    for _ in range(200):
        key, block = g.bytes(klen), g.bytes(16)
        assert oracle.decrypt_block(key, oracle.encrypt_block(key, block)) == block


# --------------------------------------------------------------------------
# Counter mode, SP 800-38A Sec. 6.5 + inc32
# --------------------------------------------------------------------------

LENGTHS = [0, 1, 15, 16, 17, 31, 32, 33, 4095, 4096, 4097, 65536 + 5]


def test_counter_block_layout():
    nonce = bytes(range(12))
    assert oracle.counter_block(nonce, 1, 0) == nonce + b"\x00\x00\x00\x01"
    assert oracle.counter_block(nonce, 0x01020304, 0) == nonce + b"\x01\x02\x03\x04"
    assert oracle.counter_block(nonce, 0xFFFFFFFF, 1) == nonce + b"\x00\x00\x00\x00"
    assert oracle.counter_block(nonce, 0xFFFFFFFE, 5) == nonce + b"\x00\x00\x00\x03"


@needs_openssl
@pytest.mark.parametrize("klen", [16, 32])
@pytest.mark.parametrize("length", LENGTHS)
def test_ctr_matches_openssl(klen, length):
    g = np.random.default_rng(1000 * klen + length)
    key, nonce, data = g.bytes(klen), g.bytes(12), g.bytes(length)
    ctr0 = int(g.integers(0, 1 << 32))
    assert bytes(oracle.ctr(key, nonce, ctr0, data)) == _openssl.ctr_inc32(key, nonce, ctr0, data)


@needs_openssl
@pytest.mark.parametrize("ctr0", [0xFFFFFFFF, 0xFFFFFFFE, 0xFFFFFFF0, 0xFFFFFFC0])
def test_ctr_wrap_matches_split_openssl(ctr0):
    g = np.random.default_rng(ctr0 & 0xFFFF)
    for klen in (16, 32):
        key, nonce, data = g.bytes(klen), g.bytes(12), g.bytes(16 * 100 + 7)
        assert bytes(oracle.ctr(key, nonce, ctr0, data)) == _openssl.ctr_inc32(key, nonce, ctr0, data)


def test_ctr_wrap_keeps_nonce():
    """After the wrap the block uses counter 0 with the same nonce."""
    g = np.random.default_rng(9)
    key, nonce = g.bytes(16), g.bytes(12)
    ks = oracle.ctr(key, nonce, 0xFFFFFFFF, bytes(32))
    assert bytes(ks[16:]) == oracle.encrypt_block(key, nonce + b"\x00\x00\x00\x00")
    assert bytes(ks[:16]) == oracle.encrypt_block(key, nonce + b"\xff\xff\xff\xff")


@pytest.mark.parametrize("klen", [16, 32])
def test_ctr_involution(klen):
    g = np.random.default_rng(31 + klen)
    key, nonce, data = g.bytes(klen), g.bytes(12), g.bytes(10_000)
    c = oracle.ctr(key, nonce, 77, data)
    assert bytes(oracle.ctr(key, nonce, 77, c)) == data


def test_ctr_split_invariance():
    g = np.random.default_rng(41)
    key, nonce, data = g.bytes(32), g.bytes(12), g.bytes(16 * 300 + 9)
    ctr0 = 0xFFFFFF00
    whole = oracle.ctr(key, nonce, ctr0, data)
    for cut_blocks in (0, 1, 17, 256, 300):
        a = oracle.ctr(key, nonce, ctr0, data[:16 * cut_blocks])
        b = oracle.ctr(key, nonce, (ctr0 + cut_blocks) & 0xFFFFFFFF, data[16 * cut_blocks:])
        assert bytes(whole) == bytes(a) + bytes(b)


def test_ctr_keystream_block_identity():
    g = np.random.default_rng(51)
    key, nonce = g.bytes(16), g.bytes(12)
    ks = oracle.ctr(key, nonce, 12345, bytes(16 * 40))
    for j in range(40):
        expect = oracle.encrypt_block(key, oracle.counter_block(nonce, 12345, j))
        assert bytes(ks[16 * j:16 * j + 16]) == expect


def test_ctr_partial_block_uses_prefix():
    g = np.random.default_rng(61)
    key, nonce = g.bytes(16), g.bytes(12)
    full = oracle.ctr(key, nonce, 3, bytes(48))
    for n in range(1, 48):
        assert bytes(oracle.ctr(key, nonce, 3, bytes(n))) == bytes(full[:n])


def test_ctr_multithreaded_equals_single():
    g = np.random.default_rng(71)
    key, nonce, data = g.bytes(32), g.bytes(12), g.bytes(16 * 5000 + 3)
    one = oracle.ctr(key, nonce, 0xFFFFF000, data)
    for t in (2, 3, 7, 0):
        assert bytes(oracle.ctr(key, nonce, 0xFFFFF000, data, threads=t)) == bytes(one)


def test_ctr_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.ctr(b"\x00" * 15, b"\x00" * 12, 0, b"")
    with pytest.raises(ValueError):
        oracle.ctr(b"\x00" * 16, b"\x00" * 11, 0, b"")
