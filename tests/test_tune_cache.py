"""The shipped autotuner cache (paper_2607_02630_amd/tune_cache.json) is
well-formed and names only shapes the library launches (no GPU).

The library reads this file beside libaesctr.so and takes an entry's shape
for the message sizes it was tuned at, so a bad entry would turn every call
of that size into an AES_EINVAL.  Each entry is checked against the launch
constraints the kernels state: T-table workgroups of 256/512/1024 threads and
its three LDS layouts, first-chunk modes 1 and 2 only where they are built
(1-2 blocks per lane, up to 512 threads; mode 1 with two tables of 32
copies), 64-256 threads for the two table-free kernels and one block per lane
for the vector-permute one; the batch entry's tile constants.  The sweep
sizes of every kernel and key size each have exactly one entry.
"""
from __future__ import annotations

import json
import os

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CACHE = os.path.join(ROOT, "paper_2607_02630_amd", "tune_cache.json")


def load():
    with open(CACHE) as f:
        return json.load(f)


def test_cache_header():
    c = load()
    assert isinstance(c.get("generated"), str) and c["generated"]
    assert isinstance(c.get("entries"), list) and c["entries"]


def first_mode_ok(mode, copies, tables, bpl, wg):
    if mode == 0:
        return True
    if bpl > 2 or wg > 512:
        return False
    return mode == 2 or (mode == 1 and copies == 32 and tables == 2)


def test_every_entry_is_a_launchable_shape():
    for e in load()["entries"]:
        v = e["variant"]
        assert v in (1, 2, 3, 10), e
        if v == 10:
            assert e["tiles_per_cu"] > 0, e
            assert e["max_tile_bytes"] % 2048 == 0 and 2048 <= e["max_tile_bytes"] <= 256 * 1024, e
            assert e["bpl"] in (1, 2), e
            continue
        assert e["key_bits"] in (128, 256), e
        assert 12 <= e["size_log2"] <= 28, e
        assert e["grid_per_cu"] in (1, 2, 4), e
        if v == 1:
            assert e["wg"] in (256, 512, 1024), e
            assert e["bpl"] in (1, 2, 4), e
            assert (e["copies"], e["tables"]) in ((32, 4), (64, 2), (32, 2)), e
            assert first_mode_ok(e.get("first", 0), e["copies"], e["tables"], e["bpl"], e["wg"]), e
        else:
            assert e["wg"] in (64, 128, 192, 256), e
            assert (e["copies"], e["tables"]) == (0, 0), e
            if v == 3:
                assert e["bpl"] == 1, e


def test_each_sweep_size_has_one_entry():
    entries = load()["entries"]
    keys = [(e["variant"], e["key_bits"], e["size_log2"]) for e in entries if e["variant"] != 10]
    assert len(keys) == len(set(keys))
    for v in (1, 2, 3):
        for bits in (128, 256):
            for size in W.SWEEP_SIZES + [W.BIG_SIZE]:
                assert (v, bits, size.bit_length() - 1) in keys, (v, bits, size)
    assert sum(e["variant"] == 10 for e in entries) == 1
