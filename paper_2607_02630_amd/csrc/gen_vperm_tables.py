#!/usr/bin/env python3
"""Generate the nibble tables of the vector-permute AES kernel (ctr_vperm.hip).

The kernel computes the AES S-box without memory lookups: its only table
lookups are 16-entry lookups done with the byte permute instruction
v_perm_b32, in the spirit of Hamburg, "Accelerating AES with vector permute
instructions" (CHES 2009), which inverts in GF(2^8) through its subfield
GF(2^4) with 4-bit table lookups.  Every table here is derived from the field
arithmetic (nothing is typed in):

1. GF(16) = GF(2)[z]/(z^4 + z + 1); T = GF(16)[Y]/(Y^2 + Y + nu) with nu of
   absolute trace 1 (so the quadratic is irreducible), and a = 1/nu.  The AES
   field GF(2)[x]/(x^8 + x^4 + x^3 + x + 1) maps into T by the GF(2)-linear
   isomorphism phi sending x to a root beta of the AES polynomial.
2. A state byte s is kept as two nibbles (i, k) with phi(s) = i*(a*Y) + k.
   With D = a*i^2 + a*i*k + k^2 (the norm of phi(s)), j = i + k and the
   projective conventions 1/0 = inf, 1/inf = 0, inf + v = inf, the chain
        ia = 1/i + a/k,  ja = 1/j + a/k,  io = 1/ia + j,  jo = 1/ja + i
   gives 1/io = (a*i + k)/D and 1/jo = ((1 + a)(a*i + k) + a*a*i)/D, from
   which the two coordinates of phi(s)^-1 = (a*i/D)*Y + (a*i + k)/D follow
   as a sum F(io) + G(jo) of two functions of one nibble each:
        F(io) = ((1 + a)/a)/io * Y + 1/io,    G(jo) = (1/a)/jo * Y
   (F and G are 0 at 0 and at inf).  The generator checks this on all 256
   inputs.  Any GF(2)-linear function of s^-1 (the S-box's affine map
   without its constant, times a MixColumns coefficient, projected onto a
   nibble of the (i, k) representation or onto standard bits) is then
   F'(io) xor G'(jo) for tables F', G'.
3. Encoding in a byte lane.  A nibble n is stored as the byte
   E(n) = (n & 7) | (n >> 3) << 7, so XOR of encodings is the encoding of the
   XOR; inf is 0x40 (bit 6), which no XOR with a finite nibble clears.  A
   16-entry lookup of byte lanes e is
        perm(W1, W0, e) xor perm(W3, W2, e xor 0x80)
   with W0..W3 holding the complemented table entries 0-3, 4-7, 8-11, 12-15:
   for a finite e one permute selects ~T[e] and the other (selector >= 128)
   gives 0xff, so their XOR is T[e]; for inf both selectors are >= 13 and
   give 0xff, so the lookup returns 0.
4. The S-box's constant {63} is not in any table (a lookup of inf must give
   0): MixColumns maps a column of four equal bytes c to itself, so the
   constant is added to every round key after round 0 instead.

Output: vperm_tables.inc with the table words, the byte -> (E(i), E(k))
conversion for round keys and nonce bytes, and the chosen nu and beta.

Usage: python gen_vperm_tables.py [--out vperm_tables.inc]
"""
from __future__ import annotations

import argparse
import os

INF = 16                # a nibble value outside GF(16)
INF_BYTE = 0x40


# --------------------------------------------------------------------------
# GF(16), the tower T and the AES field
# --------------------------------------------------------------------------

def g16_mul(a: int, b: int) -> int:
    r = 0
    for _ in range(4):
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a & 0x10:
            a ^= 0x13
    return r


G16_INV = [0] + [next(b for b in range(1, 16) if g16_mul(a, b) == 1) for a in range(1, 16)]


def g16_trace(v: int) -> int:
    t, s = v, v
    for _ in range(3):
        t = g16_mul(t, t)
        s ^= t
    return s


def t_mul(x, y, nu):
    """(h1 Y + l1)(h2 Y + l2) with Y^2 = Y + nu."""
    h1, l1 = x
    h2, l2 = y
    hh = g16_mul(h1, h2)
    return (hh ^ g16_mul(h1, l2) ^ g16_mul(h2, l1), g16_mul(hh, nu) ^ g16_mul(l1, l2))


def t_add(x, y):
    return (x[0] ^ y[0], x[1] ^ y[1])


def t_pow(x, e, nu):
    r = (0, 1)
    for _ in range(e):
        r = t_mul(r, x, nu)
    return r


def t_inv_table(nu):
    elems = [(h, l) for h in range(16) for l in range(16)]
    inv = {(0, 0): (0, 0)}
    for x in elems[1:]:
        inv[x] = next(y for y in elems if t_mul(x, y, nu) == (0, 1))
    return inv


def aes_mul(a: int, b: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        if a & 0x100:
            a ^= 0x11B
        b >>= 1
    return r


def aes_affine_linear(b: int) -> int:
    """FIPS-197 Sec. 5.1.1 affine map without its constant {63}."""
    out = 0
    for i in range(8):
        bit = 0
        for d in (0, 4, 5, 6, 7):
            bit ^= (b >> ((i + d) % 8)) & 1
        out |= bit << i
    return out


def aes_sbox(v: int) -> int:
    inv = 0 if v == 0 else next(y for y in range(1, 256) if aes_mul(v, y) == 1)
    return aes_affine_linear(inv) ^ 0x63


# --------------------------------------------------------------------------
# The representation
# --------------------------------------------------------------------------

class Rep:
    def __init__(self, nu: int, beta_index: int = 0):
        assert g16_trace(nu) & 1
        self.nu = nu
        self.a = G16_INV[nu]
        elems = [(h, l) for h in range(16) for l in range(16)]

        def aes_poly(t):
            acc = (0, 0)
            for e in (8, 4, 3, 1, 0):
                acc = t_add(acc, t_pow(t, e, nu))
            return acc

        roots = [t for t in elems if aes_poly(t) == (0, 0)]
        assert len(roots) == 8
        self.beta = roots[beta_index]
        # phi(byte) = sum over bits m of beta^m
        pw = [t_pow(self.beta, m, nu) for m in range(8)]
        self.phi = []
        for v in range(256):
            acc = (0, 0)
            for m in range(8):
                if (v >> m) & 1:
                    acc = t_add(acc, pw[m])
            self.phi.append(acc)
        assert len(set(self.phi)) == 256
        self.phi_inv = {t: v for v, t in enumerate(self.phi)}
        self.tinv = t_inv_table(nu)

    def parts(self, v: int):
        """(i, k) of byte v: phi(v) = i*(a*Y) + k."""
        h, l = self.phi[v]
        return g16_mul(h, self.nu), l

    def from_parts(self, i: int, k: int) -> int:
        return self.phi_inv[(g16_mul(self.a, i), k)]

    # projective nibble arithmetic of the chain
    @staticmethod
    def pinv(n):
        if n == INF:
            return 0
        if n == 0:
            return INF
        return G16_INV[n]

    @staticmethod
    def pxor(x, y):
        return INF if INF in (x, y) else x ^ y

    def adiv(self, k):
        return INF if k == 0 else g16_mul(self.a, G16_INV[k])

    def chain(self, i, k):
        j = i ^ k
        ak = self.adiv(k)
        ia = self.pxor(self.pinv(i), ak)
        ja = self.pxor(self.pinv(j), ak)
        io = self.pxor(self.pinv(ia), j)
        jo = self.pxor(self.pinv(ja), i)
        return io, jo

    def F(self, io):
        """Tower element F(io) (0 at 0 and inf)."""
        if io in (0, INF):
            return (0, 0)
        r = G16_INV[io]
        return (g16_mul(g16_mul(1 ^ self.a, G16_INV[self.a]), r), r)

    def G(self, jo):
        if jo in (0, INF):
            return (0, 0)
        return (g16_mul(G16_INV[self.a], G16_INV[jo]), 0)

    def check_inverse(self):
        for v in range(256):
            i, k = self.parts(v)
            io, jo = self.chain(i, k)
            got = t_add(self.F(io), self.G(jo))
            assert got == self.tinv[self.phi[v]], v


# --------------------------------------------------------------------------
# Tables
# --------------------------------------------------------------------------

def enc(n: int) -> int:
    if n == INF:
        return INF_BYTE
    return (n & 7) | ((n >> 3) << 7)


def table_words(t):
    """16 byte values -> 4 words of complemented entries (W0..W3)."""
    assert len(t) == 16 and all(0 <= v < 256 for v in t)
    c = [(~v) & 0xFF for v in t]
    return [c[4 * w] | c[4 * w + 1] << 8 | c[4 * w + 2] << 16 | c[4 * w + 3] << 24 for w in range(4)]


def output_tables(rep: Rep, fn):
    """Tables F', G' (16 entries each) with fn(s^-1 as tower element) =
    F'[io] xor G'[jo]; fn is GF(2)-linear from a tower element to a byte."""
    tf = [fn(rep.F(n)) for n in range(16)]
    tg = [fn(rep.G(n)) for n in range(16)]
    return tf, tg


def build(nu: int, beta_index: int):
    rep = Rep(nu, beta_index)
    rep.check_inverse()
    inv = [enc(rep.pinv(n)) for n in range(16)]
    adiv = [enc(rep.adiv(n)) for n in range(16)]

    def lin_of_inverse(t, mult):
        """Byte mult * A_lin(phi^-1(t)) (t: tower element of s^-1)."""
        return aes_mul(mult, aes_affine_linear(rep.phi_inv[t]))

    tables = {"inv": inv, "adiv": adiv}
    for name, mult in (("s", 1), ("d", 2)):
        for part in ("i", "k"):
            idx = 0 if part == "i" else 1
            fn = (lambda t, m=mult, p=idx: enc(rep.parts(lin_of_inverse(t, m))[p]))
            tf, tg = output_tables(rep, fn)
            tables[f"{name}{part}_f"] = tf
            tables[f"{name}{part}_g"] = tg
    # Final round: standard bytes of A_lin(s^-1).
    tf, tg = output_tables(rep, lambda t: lin_of_inverse(t, 1))
    tables["out_f"], tables["out_g"] = tf, tg
    # Standard nibble -> parts: byte v = lo | hi << 4.
    for part in ("i", "k"):
        idx = 0 if part == "i" else 1
        tables[f"cv{part}_lo"] = [enc(rep.parts(n)[idx]) for n in range(16)]
        tables[f"cv{part}_hi"] = [enc(rep.parts(n << 4)[idx]) for n in range(16)]
    to_parts = [enc(rep.parts(v)[0]) | enc(rep.parts(v)[1]) << 8 for v in range(256)]
    return rep, tables, to_parts


# --------------------------------------------------------------------------
# Reference evaluation of one round at the value level (self-check)
# --------------------------------------------------------------------------

def lookup(table, n):
    return 0 if n == INF_BYTE or (n & INF_BYTE) else table[(n & 7) | ((n >> 7) << 3)]


def sbox_via_tables(tables, to_parts, v):
    ei, ek = to_parts[v] & 0xFF, to_parts[v] >> 8
    ej = ei ^ ek
    ak = lookup(tables["adiv"], ek)
    ia = lookup(tables["inv"], ei) ^ ak
    ja = lookup(tables["inv"], ej) ^ ak
    io = lookup(tables["inv"], ia) ^ ej
    jo = lookup(tables["inv"], ja) ^ ei
    return lookup(tables["out_f"], io) ^ lookup(tables["out_g"], jo) ^ 0x63


def emit(rep, tables, to_parts, path):
    lines = ["// vperm_tables.inc -- generated by gen_vperm_tables.py; do not edit.",
             f"// GF(16) = GF(2)[z]/(z^4+z+1); T = GF(16)[Y]/(Y^2+Y+nu), nu = {rep.nu:#x}, a = 1/nu = {rep.a:#x};",
             f"// beta = {rep.beta[0]:#x}*Y + {rep.beta[1]:#x} (root of the AES polynomial in T).",
             "// Each table: four words of complemented entries 0-3, 4-7, 8-11, 12-15 (byte e of",
             "// word w is ~T[4w + e]); a lookup is perm(W1, W0, e) ^ perm(W3, W2, e ^ 0x80).",
             ""]
    order = ["inv", "adiv", "si_f", "si_g", "sk_f", "sk_g", "di_f", "di_g", "dk_f", "dk_g", "out_f", "out_g",
             "cvi_lo", "cvi_hi", "cvk_lo", "cvk_hi"]
    for name in order:
        w = table_words(tables[name])
        lines.append(f"constexpr uint32_t kVp_{name}[4] = {{{', '.join(f'0x{x:08x}u' for x in w)}}};")
    lines.append("")
    lines.append("// Byte v -> E(i) | E(k) << 8 with phi(v) = i*(a*Y) + k.")
    rows = []
    for r in range(0, 256, 8):
        rows.append("    " + ", ".join(f"0x{to_parts[v]:04x}" for v in range(r, r + 8)) + ",")
    lines.append("constexpr uint16_t kVpToParts[256] = {")
    lines.extend(rows)
    lines.append("};")
    lines.append(f"constexpr uint32_t kVpInf = 0x{INF_BYTE:02x}u;")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "vperm_tables.inc"))
    ap.add_argument("--nu", type=int, default=0, help="GF(16) constant of the tower (default: smallest valid)")
    args = ap.parse_args()
    nu = args.nu or next(v for v in range(2, 16) if g16_trace(v) & 1)
    rep, tables, to_parts = build(nu, 0)
    for v in range(256):
        assert sbox_via_tables(tables, to_parts, v) == aes_sbox(v), v
    emit(rep, tables, to_parts, args.out)
    print(f"wrote {args.out} (nu = {nu:#x}, beta = {rep.beta})")


if __name__ == "__main__":
    main()
