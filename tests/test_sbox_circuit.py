"""The bitsliced kernel's S-box circuit equals the oracle's S-box (no GPU).

sbox_circuit.inc is evaluated here as written: each line is one 3-input
boolean function v_bitop3_b32(a, b, c, T), whose value for inputs (a, b, c)
is bit (a<<2 | b<<1 | c) of T.  The 8 input words carry, bit-sliced, all 256
byte values; the 8 outputs must carry FIPS-197's S-box of each.
"""
from __future__ import annotations

import os
import re

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "paper_2607_02630_amd", "csrc", "sbox_circuit.inc")
FULL = (1 << 256) - 1


def bitop3(a: int, b: int, c: int, t: int) -> int:
    out = 0
    for idx in range(8):
        if (t >> idx) & 1:
            term = FULL
            term &= a if idx & 4 else ~a & FULL
            term &= b if idx & 2 else ~b & FULL
            term &= c if idx & 1 else ~c & FULL
            out |= term
    return out


def run_circuit(text: str) -> list[int]:
    env = {f"x[{b}]": sum(((v >> b) & 1) << v for v in range(256)) for b in range(8)}
    pat = re.compile(r"const uint32_t (\w+) = bitop3\(([^,]+), ([^,]+), ([^,]+), (0x[0-9a-f]+)\);")
    outs = {}
    n = 0
    for line in text.splitlines():
        m = pat.search(line)
        if m:
            name, a, b, c, t = m.groups()
            env[name] = bitop3(env[a.strip()], env[b.strip()], env[c.strip()], int(t, 16))
            n += 1
            continue
        m = re.search(r"x\[(\d)\] = (\w+);", line)
        if m:
            outs[int(m.group(1))] = env[m.group(2)]
    assert sorted(outs) == list(range(8)) and n > 0
    return [sum(((outs[b] >> v) & 1) << b for b in range(8)) for v in range(256)]


def test_circuit_is_the_sbox():
    got = run_circuit(open(INC).read())
    assert got == list(oracle.sbox())


def test_circuit_mutation_is_caught():
    """Flipping one truth-table bit of any node changes the S-box."""
    text = open(INC).read()
    lines = [l for l in text.splitlines() if "const uint32_t" in l]
    for l in lines[::7]:
        t = re.search(r"(0x[0-9a-f]+)\);", l).group(1)
        bad = l.replace(t + ");", f"0x{int(t, 16) ^ 0x01:02x});")
        assert run_circuit(text.replace(l, bad)) != list(oracle.sbox())
