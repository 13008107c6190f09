"""The vector-permute kernel's tables and round sequence, emulated on the CPU.

vperm_tables.inc is read as written and the kernel's per-block sequence is
run word by word with the byte-permute semantics of v_perm_b32 (bytes 0-3 of
the pair are the second source, 4-7 the first; selector bytes 0-7 pick a
byte, 8-11 replicate a sign bit, 12 gives 0x00 and 13 or more 0xff).  The
result must equal the oracle's FIPS-197 cipher for AES-128 and AES-256 on
random keys and on every counter-block shape the kernel sees; a flipped
table bit must be caught.  No GPU.
"""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2607_02630_amd", "csrc", "vperm_tables.inc")
C = 0x80808080
M32 = 0xFFFFFFFF


def parse(text: str):
    tabs = {m.group(1): [int(x.rstrip("u"), 16) for x in m.group(2).split(",")]
            for m in re.finditer(r"kVp_(\w+)\[4\] = \{([^}]*)\}", text)}
    body = re.search(r"kVpToParts\[256\] = \{([^}]*)\}", text).group(1)
    to_parts = [int(x, 16) for x in body.replace("\n", " ").split(",") if x.strip()]
    assert len(to_parts) == 256
    return tabs, to_parts


def vperm(s0: int, s1: int, sel: int) -> int:
    pair = [(s1 >> (8 * b)) & 0xFF for b in range(4)] + [(s0 >> (8 * b)) & 0xFF for b in range(4)]
    out = 0
    for b in range(4):
        s = (sel >> (8 * b)) & 0xFF
        if s >= 13:
            v = 0xFF
        elif s == 12:
            v = 0
        elif s >= 8:
            v = 0xFF if pair[(s - 8) * 2 + 1] & 0x80 else 0
        else:
            v = pair[s]
        out |= v << (8 * b)
    return out


def look(t, e: int) -> int:
    return vperm(t[1], t[0], e) ^ vperm(t[3], t[2], e ^ C)


def rotr(x: int, n: int) -> int:
    return ((x >> n) | (x << (32 - n))) & M32 if n else x


def mix_coef(r: int, rp: int) -> int:
    """MixColumns coefficient of row rp's byte in output row r."""
    return 2 if rp == r else 3 if rp == (r + 1) % 4 else 1


def prep(key: bytes, nonce: bytes, to_parts):
    """Round-key material as the kernel takes it: per round t >= 2 and row r
    the parts words of (round key t) xor {63}; for round 1 the constant part
    of each output row (the nonce columns' MixColumns terms, rk1, and the
    {63} fold of the counter term); the final round's standard bytes; x0."""
    nr, w = oracle.expand(key)
    rk = [[(w[4 * t + c] >> (24 - 8 * r)) & 0xFF for c in range(4) for r in range(4)] for t in range(nr + 1)]
    # rk[t][4c + r] = byte r of column c of round key t

    def parts_word(vals, which):
        return sum(((to_parts[v] >> (8 * which)) & 0xFF) << (8 * c) for c, v in enumerate(vals))

    rki = [[parts_word([rk[t][4 * c + r] ^ 0x63 for c in range(4)], 0) for r in range(4)] for t in range(nr + 1)]
    rkk = [[parts_word([rk[t][4 * c + r] ^ 0x63 for c in range(4)], 1) for r in range(4)] for t in range(nr + 1)]
    rkn = [sum((rk[nr][4 * c + r] ^ 0x63) << (8 * c) for c in range(4)) for r in range(4)]
    # Round 1 (FIPS-197 Sec. 5.1): after ShiftRows, state byte (r', c) is
    # round-0 byte (r', c + r'), and output column c's counter byte is the
    # one of row 3 - c.  Everything else of output byte (r, c) is constant.
    sbox = [int(v) for v in oracle.sbox()]
    state0 = [[nonce[4 * c + r] ^ rk[0][4 * c + r] for c in range(3)] for r in range(4)]
    const1 = [[0] * 4 for _ in range(4)]
    for r in range(4):
        for c in range(4):
            v = rk[1][4 * c + r] ^ oracle.gf_mul(mix_coef(r, 3 - c), 0x63)
            for rp in range(4):
                if rp != 3 - c:
                    v ^= oracle.gf_mul(mix_coef(r, rp), sbox[state0[rp][(c + rp) % 4]])
            const1[r][c] = v
    rki[1] = [parts_word(const1[r], 0) for r in range(4)]
    rkk[1] = [parts_word(const1[r], 1) for r in range(4)]
    x0 = sum(rk[0][12 + r] << (8 * r) for r in range(4))
    return nr, rki, rkk, rkn, x0


def row1_selectors(r: int):
    """v_perm_b32 selectors of round-1 output row r: byte c takes coefficient
    mix_coef(r, 3 - c) times byte 3 - c of S (from S or T = 3S) or of D = 2S."""
    sel = dsel = 0
    for c in range(4):
        rp, k = 3 - c, mix_coef(r, 3 - c)
        sel |= (rp if k == 1 else 4 + rp if k == 3 else 12) << (8 * c)
        dsel |= (rp if k == 2 else 12) << (8 * c)
    return sel, dsel


def chain(T, I: int, K: int):
    ak = look(T["adiv"], K)
    j = I ^ K
    ia = look(T["inv"], I) ^ ak
    ja = look(T["inv"], j) ^ ak
    return look(T["inv"], ia) ^ j, look(T["inv"], ja) ^ I


def encrypt(tabs, key_mat, ctr: int) -> bytes:
    nr, rki, rkk, rkn, x0 = key_mat
    T = tabs
    bswap = vperm(ctr, ctr, 0x00010203)
    X = bswap ^ x0
    lo = (X & 0x07070707) | ((X << 4) & C)
    hi = ((X >> 4) & 0x07070707) | (X & C)
    XI = look(T["cvi_lo"], lo) ^ look(T["cvi_hi"], hi)
    XK = look(T["cvk_lo"], lo) ^ look(T["cvk_hi"], hi)
    # Round 1 from the counter column alone.
    io1, jo1 = chain(T, XI, XK)
    w = {name: look(T[name + "_f"], io1) ^ look(T[name + "_g"], jo1) for name in ("si", "sk", "di", "dk")}
    I, K = [], []
    for r in range(4):
        sel, dsel = row1_selectors(r)
        I.append(vperm(w["si"] ^ w["di"], w["si"], sel) ^ vperm(w["di"], w["di"], dsel) ^ rki[1][r])
        K.append(vperm(w["sk"] ^ w["dk"], w["sk"], sel) ^ vperm(w["dk"], w["dk"], dsel) ^ rkk[1][r])
    for t in range(2, nr + 1):
        I = [rotr(I[r], 8 * r) for r in range(4)]
        K = [rotr(K[r], 8 * r) for r in range(4)]
        io, jo = [], []
        for r in range(4):
            a, b = chain(T, I[r], K[r])
            io.append(a)
            jo.append(b)
        if t < nr:
            out = {}
            for name in ("si", "sk", "di", "dk"):
                out[name] = [look(T[name + "_f"], io[r]) ^ look(T[name + "_g"], jo[r]) for r in range(4)]
            I = [out["di"][r] ^ out["di"][(r + 1) % 4] ^ out["si"][(r + 1) % 4] ^ out["si"][(r + 2) % 4]
                 ^ out["si"][(r + 3) % 4] ^ rki[t][r] for r in range(4)]
            K = [out["dk"][r] ^ out["dk"][(r + 1) % 4] ^ out["sk"][(r + 1) % 4] ^ out["sk"][(r + 2) % 4]
                 ^ out["sk"][(r + 3) % 4] ^ rkk[t][r] for r in range(4)]
        else:
            rows = [look(T["out_f"], io[r]) ^ look(T["out_g"], jo[r]) ^ rkn[r] for r in range(4)]
            return bytes((rows[r] >> (8 * c)) & 0xFF for c in range(4) for r in range(4))


@pytest.fixture(scope="module")
def tables():
    return parse(open(INC).read())


@pytest.mark.parametrize("klen", [16, 32])
def test_emulated_kernel_equals_the_oracle(tables, klen):
    tabs, to_parts = tables
    g = np.random.default_rng(klen)
    for _ in range(6):
        key, nonce = g.bytes(klen), g.bytes(12)
        km = prep(key, nonce, to_parts)
        for ctr in [0, 1, 255, 256, 0xFFFFFFFF, 0x01020304] + [int(x) for x in g.integers(0, 1 << 32, 4)]:
            block = nonce + ctr.to_bytes(4, "big")
            assert encrypt(tabs, km, ctr) == oracle.encrypt_block(key, block), (key.hex(), ctr)


def test_every_state_byte_value_passes_the_sbox_sequence(tables):
    """All 256 byte values at every position of one full round: a key whose
    round-0 state sweeps the counter column through 0..255."""
    tabs, to_parts = tables
    key, nonce = bytes(range(16)), bytes(range(100, 112))
    km = prep(key, nonce, to_parts)
    for v in range(256):
        ctr = v * 0x01010101
        assert encrypt(tabs, km, ctr) == oracle.encrypt_block(key, nonce + ctr.to_bytes(4, "big"))


def test_flipped_table_bit_is_caught(tables):
    """A flipped bit in any table entry the sequence reads changes some
    output.  Entry 0 of the output tables is never read: io and jo are never
    the nibble 0 (1/io = 0 would need a zero norm, i.e. a zero state byte,
    whose chain gives inf for both instead)."""
    tabs, to_parts = tables
    key, nonce = bytes(range(32)), bytes(12)
    km = prep(key, nonce, to_parts)
    ctrs = list(range(0, 1 << 32, (1 << 32) // 97))[:97]
    for name in sorted(tabs):
        for w in range(4):
            for bit in ((8, 13, 31) if w == 0 and name.endswith(("_f", "_g")) else (0, 13, 31)):
                bad = {k: list(v) for k, v in tabs.items()}
                bad[name][w] ^= 1 << bit
                assert any(encrypt(bad, km, c) != oracle.encrypt_block(key, nonce + c.to_bytes(4, "big"))
                           for c in ctrs), (name, w, bit)
