"""GPU parity of aes_ctr_crypt against the CPU oracle (bit-exact).

Covers the 1 MiB AES-128 workload, the AES-128 and AES-256 sweeps at full
size (4 KiB .. 8 MiB and 256 MiB, checked through oracle-written digests),
every kernel variant and launch shape on inputs spanning many workgroup
chunks plus a ragged tail, odd lengths, unaligned and in-place buffers, and
counter wrap-around.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import golden, log, sha256, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

A = None


def lib():
    global A
    if A is None:
        import paper_2607_02630_amd as mod
        A = mod
    return A


def gpu_crypt(key: bytes, nonce: bytes, ctr0: int, data: np.ndarray, cfg=None,
              in_off: int = 0, out_off: int = 0) -> np.ndarray:
    torch = torch_cuda()
    L = lib()
    s = L.aes_expand_key(key)
    _, src = to_dev(data, offset=in_off)
    _, dst = to_dev(np.zeros(len(data), np.uint8), offset=out_off)
    L.aes_ctr_crypt(s, nonce, ctr0, src, dst, length=len(data), cfg=cfg)
    torch.cuda.synchronize()
    return to_host(dst)


# Every LDS layout (copies, tables): four tables x 32, two x 64, two x 32.
TT_SHAPES = [dict(variant=1, lds_copies=c, lds_tables=t, blocks_per_lane=b, wg_size=w)
             for c, t in ((32, 4), (64, 2), (32, 2)) for b in (1, 2, 4) for w in (256, 1024)]
# The first-chunk modes (1 per-wave group constants, 2 rounds 1-2 in full,
# 3 wave 0 for the workgroup) on the shapes built with them.
FIRST_SHAPES = ([dict(variant=1, lds_copies=32, lds_tables=2, blocks_per_lane=b, wg_size=w, wave_groups=m)
                 for b in (1, 2) for w in (256, 512) for m in (1, 2, 3)]
                + [dict(variant=1, lds_copies=32, lds_tables=4, blocks_per_lane=1, wg_size=256, wave_groups=2)])
BS_SHAPES = [dict(variant=2, wg_size=w) for w in (64, 256)]
VP_SHAPES = [dict(variant=3, wg_size=w) for w in (64, 256)]
SHAPES = TT_SHAPES + FIRST_SHAPES + BS_SHAPES + VP_SHAPES


def shape_id(kw):
    short = {"lds_copies": "c", "lds_tables": "t", "blocks_per_lane": "b", "wg_size": "w", "wave_groups": "g"}
    name = {1: "tt", 2: "bs", 3: "vp"}[kw["variant"]]
    return name + "".join(f"-{short[k]}{v}" for k, v in kw.items() if k != "variant")


def test_single_1mib_matches_oracle():
    s = W.single_1mib()
    log("single 1 MiB AES-128")
    got = gpu_crypt(s.key, s.nonce, s.ctr0, s.data)
    g = golden()["single_1mib"]
    assert sha256(got) == g["sha256"]
    ref = oracle.ctr(s.key, s.nonce, s.ctr0, s.data, threads=0)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("variant", [0, 2, 3], ids=["default", "bs", "vp"])
@pytest.mark.parametrize("bits", [128, 256])
@pytest.mark.parametrize("size", W.SWEEP_SIZES + [W.BIG_SIZE])
def test_sweep_full_size_digest(bits, size, variant):
    """Every sweep size, in the default launch shape and in the bitsliced and
    vector-permute kernels', against the oracle-written digest (the
    configurations the benchmark's sweep times)."""
    key, nonce = W.sweep_key(bits)
    data = W.sweep_payload(size, bits)
    log(f"sweep AES-{bits} {size} B variant {variant}")
    cfg = lib().launch_cfg(variant=variant) if variant else None
    got = gpu_crypt(key, nonce, 1, data, cfg=cfg)
    assert sha256(got) == golden()["sweep"][f"{bits}/{size}"]


@pytest.mark.parametrize("ctr0", [0xFFFFF000, 0xFFFFF0F7], ids=["aligned", "midgroup"])
@pytest.mark.parametrize("kw", SHAPES, ids=shape_id)
@pytest.mark.parametrize("klen", [16, 32])
def test_launch_shapes_match_oracle(kw, klen, ctr0):
    """Every launch shape, on a message of many chunks with a ragged tail
    whose counter wraps mod 2^32.  The mid-group start counter makes each
    workgroup chunk begin inside a 256-counter group, so a 4096-block chunk
    touches the most groups (17)."""
    g = np.random.default_rng(7 + klen)
    key, nonce = g.bytes(klen), g.bytes(12)
    data = W.payload(g, (1 << 19) + 16 * 37 + 5)
    ref = oracle.ctr(key, nonce, ctr0, data, threads=0)
    log(f"shape {shape_id(kw)} AES-{8 * klen} ctr0 {ctr0:#x}")
    for grid in (0, 3):     # tuned grid, and a tiny grid that loops many times
        cfg = lib().launch_cfg(grid=grid, **kw)
        got = gpu_crypt(key, nonce, ctr0, data, cfg=cfg)
        assert np.array_equal(got, ref), (kw, grid)


LENGTHS = [1, 15, 16, 17, 31, 33, 1023, 4095, 4096, 4097, 65537, (1 << 20) + 15]


@pytest.mark.parametrize("variant", [1, 2, 3], ids=["tt", "bs", "vp"])
@pytest.mark.parametrize("n", LENGTHS)
def test_lengths(variant, n):
    g = np.random.default_rng(n)
    key, nonce = g.bytes(16), g.bytes(12)
    data = W.payload(g, n)
    got = gpu_crypt(key, nonce, 5, data, cfg=lib().launch_cfg(variant=variant))
    assert np.array_equal(got, oracle.ctr(key, nonce, 5, data))


@pytest.mark.parametrize("variant", [1, 2, 3], ids=["tt", "bs", "vp"])
@pytest.mark.parametrize("offs", [(1, 0), (0, 3), (7, 7), (15, 9), (4, 8)])
def test_unaligned_buffers(variant, offs):
    g = np.random.default_rng(offs[0] * 16 + offs[1])
    key, nonce = g.bytes(32), g.bytes(12)
    data = W.payload(g, 16 * 3000 + 11)
    got = gpu_crypt(key, nonce, 9, data, cfg=lib().launch_cfg(variant=variant),
                    in_off=offs[0], out_off=offs[1])
    assert np.array_equal(got, oracle.ctr(key, nonce, 9, data))


@pytest.mark.parametrize("variant", [1, 2, 3], ids=["tt", "bs", "vp"])
def test_in_place(variant):
    torch = torch_cuda()
    g = np.random.default_rng(99)
    key, nonce = g.bytes(16), g.bytes(12)
    data = W.payload(g, 200_000 + 3)
    _, buf = to_dev(data)
    L = lib()
    L.aes_ctr_crypt(L.aes_expand_key(key), nonce, 1, buf, buf, cfg=L.launch_cfg(variant=variant))
    torch.cuda.synchronize()
    assert np.array_equal(to_host(buf), oracle.ctr(key, nonce, 1, data))


@pytest.mark.parametrize("klen", [16, 32])
@pytest.mark.parametrize("variant", [1, 2, 3], ids=["tt", "bs", "vp"])
@pytest.mark.parametrize("ctr0", [0xFFFFFFFF, 0xFFFFFF00, 0xFFFFFFF0, 0x7FFFFF00, 0x80000013, 0xC0FFEE00])
def test_counter_wrap(variant, ctr0, klen):
    """Counters that wrap mod 2^32, and counters at and above 2^31 (where a
    signed shift of the counter would corrupt its high bits)."""
    g = np.random.default_rng(ctr0 & 0xFFF)
    key, nonce = g.bytes(klen), g.bytes(12)
    data = W.payload(g, 16 * 700 + 9)
    got = gpu_crypt(key, nonce, ctr0, data, cfg=lib().launch_cfg(variant=variant))
    assert np.array_equal(got, oracle.ctr(key, nonce, ctr0, data))


@pytest.mark.parametrize("klen", [16, 32])
@pytest.mark.parametrize("size", [(8 << 20) + 5, (64 << 20) + 21], ids=["8MiB+5", "64MiB+21"])
def test_default_large_shapes_across_the_wrap(size, klen):
    """The default shapes of large launches (two workgroups per CU in the
    grid, two chunks per workgroup at 64 MiB), with the counter wrapping
    mod 2^32 in the middle of the message and a ragged tail."""
    g = np.random.default_rng(size & 0xFFFF)
    key, nonce = g.bytes(klen), g.bytes(12)
    data = W.payload(g, size)
    ctr0 = (1 << 32) - (size // 16) // 2 - 3
    log(f"AES-{8 * klen} {size} B default shape, ctr0 {ctr0:#x}")
    got = gpu_crypt(key, nonce, ctr0, data)
    assert np.array_equal(got, oracle.ctr(key, nonce, ctr0, data, threads=0))


@pytest.mark.parametrize("klen", [16, 32])
@pytest.mark.parametrize("wg", [256, 512])
@pytest.mark.parametrize("per_cu", [2, 4])
def test_per_wave_group_constants(per_cu, wg, klen):
    """Two-table shapes with two blocks per lane and at least two workgroups
    per CU, where every wave computes its first chunk's group constants
    itself: 8 MiB and a ragged tail, from a start counter inside a group,
    wrapping mod 2^32 part-way; with four workgroups per CU the buffers are
    unaligned (the byte-wise load and store path)."""
    torch = torch_cuda()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    g = np.random.default_rng(11 * wg + klen + per_cu)
    key, nonce = g.bytes(klen), g.bytes(12)
    data = W.payload(g, (8 << 20) + 16 * 37 + 5)
    ctr0 = 0xFFFFF0F7
    cfg = lib().launch_cfg(variant=1, lds_copies=32, lds_tables=2, blocks_per_lane=2, wg_size=wg,
                           grid=per_cu * cus)
    shape = lib().launch_shape(8 * klen, len(data), cfg)
    assert shape["grid"] >= 2 * cus and shape["wave_groups"] == 1, shape
    in_off, out_off = (3, 5) if per_cu == 4 else (0, 0)
    log(f"per-wave group constants: AES-{8 * klen} wg {wg} grid {shape['grid']} offsets {in_off}/{out_off}")
    got = gpu_crypt(key, nonce, ctr0, data, cfg=cfg, in_off=in_off, out_off=out_off)
    assert np.array_equal(got, oracle.ctr(key, nonce, ctr0, data, threads=0))


def test_decrypt_roundtrip_and_zero_length():
    torch = torch_cuda()
    L = lib()
    g = np.random.default_rng(5)
    key, nonce = g.bytes(32), g.bytes(12)
    data = W.payload(g, 123_457)
    s = L.aes_expand_key(key)
    _, x = to_dev(data)
    c = L.aes_ctr_crypt(s, nonce, 77, x)
    p = L.aes_ctr_crypt(s, nonce, 77, c)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(p), data)
    empty = torch.empty(0, dtype=torch.uint8, device="cuda")
    L.aes_ctr_crypt(s, nonce, 1, empty, empty)


def test_overlap_rejected_on_device():
    torch = torch_cuda()
    L = lib()
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    s = L.aes_expand_key(bytes(16))
    rc = L.lib.aes_ctr_crypt(ctypes.byref(s), bytes(12), 1, buf.data_ptr(),
                             buf.data_ptr() + 16, 1024, torch.cuda.current_stream().cuda_stream)
    assert rc == -8


RULE_CHECK = r"""
import torch
import paper_2607_02630_amd as A
cus = torch.cuda.get_device_properties(0).multi_processor_count
MiB = 1 << 20


def shape(bits, size, **kw):
    return A.launch_shape(bits, size, A.launch_cfg(**kw) if kw else None)


# The rule works in blocks per CU; these sizes are the MI355X ones (256 CUs).
scale = cus / 256
s = shape(128, int(1 * MiB * scale))
assert (s["lds_copies"], s["lds_tables"], s["wg_size"], s["blocks_per_lane"]) == (32, 2, 256, 1), s
assert s["wave_groups"] == 2, s         # one chunk per workgroup: rounds 1-2 in full
s = shape(256, int(1 * MiB * scale))
assert (s["lds_tables"], s["wg_size"], s["wave_groups"]) == (2, 256, 2), s
s = shape(128, int(2 * MiB * scale))
assert (s["wg_size"], s["blocks_per_lane"], s["wave_groups"]) == (512, 1, 2), s
s = shape(128, int(4 * MiB * scale))
assert (s["lds_tables"], s["wg_size"], s["blocks_per_lane"]) == (2, 512, 2), s
s = shape(128, int(8 * MiB * scale))
assert (s["lds_copies"], s["lds_tables"], s["wg_size"], s["blocks_per_lane"]) == (32, 2, 512, 2), s
assert s["grid"] == 2 * cus, s          # four per CU, clamped to the 2 chunks per CU there are
assert s["wave_groups"] == 1, s         # two workgroups per CU: each wave its own group constants
assert shape(128, int(4 * MiB * scale))["wave_groups"] == 2
assert shape(128, int(1 * MiB * scale), wg_size=1024)["wave_groups"] == 0   # mode 2 is built up to 512
assert shape(128, int(8 * MiB * scale), wg_size=1024)["wave_groups"] == 0
assert shape(128, int(8 * MiB * scale), lds_tables=4)["wave_groups"] == 0
s = shape(128, int(32 * MiB * scale))
assert (s["wg_size"], s["blocks_per_lane"], s["grid"]) == (512, 4, 4 * cus), s
assert shape(128, MiB, lds_copies=64)["lds_tables"] == 2
assert shape(128, MiB, lds_tables=4)["lds_tables"] == 4
assert shape(128, 8 * MiB, lds_tables=4)["lds_tables"] == 4
s = shape(128, MiB, variant=2)
assert (s["lds_copies"], s["lds_tables"]) == (0, 0), s
s = shape(128, MiB, variant=3, blocks_per_lane=4)
assert (s["variant"], s["lds_copies"], s["lds_tables"], s["blocks_per_lane"]) == (3, 0, 0, 1), s
print("rule ok")
"""


def test_default_shapes_pick_the_lds_layout_by_size(tmp_path):
    """The shape rule the library falls back on without a tune cache (run in
    a process whose cache path names no file): two T-tables (64 KiB of LDS)
    at every size, one workgroup per CU with rounds 1-2 of its one chunk in
    full up to 4 MiB, and up to four per CU (two resident) from 8 MiB;
    explicit fields override; 64 copies always mean two tables."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, AESCTR_TUNE_CACHE=str(tmp_path / "none.json"))
    r = subprocess.run([sys.executable, "-c", RULE_CHECK], cwd=root, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "rule ok" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]


def test_first_chunk_modes_on_request():
    """wave_groups on input picks the T-table kernel's first-chunk mode;
    aes_ctr_launch_shape reports it, and refuses a mode the shape is not
    built for."""
    A = lib()
    MiB = 1 << 20
    base = dict(variant=1, lds_copies=32, lds_tables=2, blocks_per_lane=1, wg_size=512)
    assert A.launch_shape(128, MiB, A.launch_cfg(wave_groups=1, **base))["wave_groups"] == 1
    assert A.launch_shape(128, MiB, A.launch_cfg(wave_groups=2, **base))["wave_groups"] == 2
    assert A.launch_shape(128, MiB, A.launch_cfg(wave_groups=3, **base))["wave_groups"] == 0
    for bad in (dict(base, blocks_per_lane=4, wave_groups=2), dict(base, wg_size=1024, wave_groups=1),
                dict(base, lds_tables=4, wave_groups=1)):
        with pytest.raises(A.AesError) as e:
            A.launch_shape(128, MiB, A.launch_cfg(**bad))
        assert e.value.status == -1, bad
        g = np.random.default_rng(3)
        key, nonce = g.bytes(16), g.bytes(12)
        with pytest.raises(A.AesError):
            gpu_crypt(key, nonce, 1, W.payload(g, 4096), cfg=A.launch_cfg(**bad))
