"""Autotuner for the launch shapes (writes tune_cache.json beside the library).

For each kernel variant, key size and message size of the sweep workloads
(4 KiB .. 8 MiB and 256 MiB), every candidate shape is run on the workload's
seeded input and its output digest is compared with the expected digest in
the file given by --golden (written by the oracle) -- a candidate that is not
bit-exact stops the run -- then timed as K launches replayed from a captured
graph over buffers larger than the Infinity Cache (replays of at least 20 ms,
median of three).  The library's own shape rule is timed first; the fastest
candidate replaces it only when at least 1% faster.  The chosen shape per
(variant, key size, size) is written to the cache, which libaesctr.so reads
(AESCTR_TUNE_CACHE or tune_cache.json next to the library).

The batch kernel's tile sizing (tiles per CU, largest tile) and blocks per
lane are tuned on the 4096-request batch workload, encrypting zero payloads
so that the output is the keystream: each candidate's sampled keystream
blocks must hash to the digest in --golden.

Usage: python -m paper_2607_02630_amd.autotune --golden PATH [--quick] [--sizes B,B,...]
       [--no-batch] [--out PATH] [--report PATH]
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MiB = 1 << 20


def _load_golden(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


def candidates(variant: int, quick: bool):
    if variant == 1:
        # LDS layouts (copies, tables): four tables x 32, two x 64, two x 32;
        # grids of one workgroup per CU, and two or four with the 64 KiB
        # layout (two fit in a CU's LDS); first-chunk modes (3 wave 0, 1
        # per-wave group constants, 2 rounds 1-2 in full) where built.
        for (c, t), b, w in itertools.product(((32, 4), (64, 2), (32, 2)), (1, 2, 4),
                                              (512, 1024) if quick else (256, 512, 1024)):
            for gm in ((1, 2, 4) if t == 2 and c == 32 else (1,)):
                modes = [3]
                if b <= 2 and w <= 512:
                    modes += [2] + ([1] if (c, t) == (32, 2) else [])
                for m in modes:
                    yield dict(variant=1, lds_copies=c, lds_tables=t, blocks_per_lane=b, wg_size=w, grid=gm,
                               wave_groups=m)
    else:
        for w, gm in itertools.product((64, 128, 256), (1, 2, 4)):
            yield dict(variant=variant, wg_size=w, grid=gm)


MIN_REPLAY_S = 0.020     # each timed replay lasts at least this long


def time_shape(torch, A, sched, nonce, ins, outs, cfg, size, repeats=3):
    """Per-launch time of a launch shape: K back-to-back launches over the
    rotating buffers, captured in a graph of at least MIN_REPLAY_S (so the
    replay's own fixed cost is spread over K launches), replayed once to
    warm up and `repeats` times timed; the median, in ms."""
    n = len(ins)

    def replay_ms(k, reps):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(k):
                A.aes_ctr_crypt(sched, nonce, 1, ins[i % n], outs[i % n], cfg=cfg)
        g.replay()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        del g
        return sorted(ts)[len(ts) // 2]

    probe = replay_ms(20, 1) / 20
    k = max(20, min(4000, math.ceil(MIN_REPLAY_S * 1e3 / max(probe, 1e-4))))
    return replay_ms(k, repeats) / k


def rule_shape(A, bits, size, variant, cus):
    """The library's own shape rule for this workload (the tune cache is
    disabled in this process), as a candidate."""
    s = A.launch_shape(bits, size, A.launch_cfg(variant=variant))
    kw = dict(variant=variant, wg_size=s["wg_size"], grid=max(1, round(s["grid"] / cus)))
    if variant == 1:
        kw.update(lds_copies=s["lds_copies"], lds_tables=s["lds_tables"], blocks_per_lane=s["blocks_per_lane"],
                  wave_groups={0: 3, 1: 1, 2: 2}[s["wave_groups"]])
    return kw


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer sizes and shapes")
    ap.add_argument("--out", default=os.path.join(HERE, "tune_cache.json"))
    ap.add_argument("--sizes", default="", help="comma-separated sweep sizes in bytes (default: all)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-kernel tile search")
    ap.add_argument("--golden", required=True,
                    help="JSON of expected digests written by the oracle (sweep digests and the "
                         "batch workload's sampled keystream digest)")
    ap.add_argument("--report", default="", help="also write every candidate's timing here (JSON)")
    args = ap.parse_args(argv)
    # Candidates are compared with the library's shape rule, not with an
    # earlier cache: no cache is read in this process.
    os.environ["AESCTR_TUNE_CACHE"] = os.path.join(HERE, "no-tune-cache-while-tuning")
    sys.path.insert(0, ROOT)
    import torch
    import workloads as W
    import paper_2607_02630_amd as A

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    golden = _load_golden(args.golden)
    gold = golden["sweep"]
    sizes = [64 * 1024, MiB, 8 * MiB, W.BIG_SIZE] if args.quick else W.SWEEP_SIZES + [W.BIG_SIZE]
    if args.sizes:
        sizes = [int(x) for x in args.sizes.split(",")]
        unknown = [x for x in sizes if f"128/{x}" not in gold]
        if unknown:
            raise SystemExit(f"no stored digests for sizes {unknown}")
    entries, report, tried = [], [], []
    for bits in (128, 256):
        key, nonce = W.sweep_key(bits)
        sched = A.aes_expand_key(key)
        for size in sizes:
            payload = W.sweep_payload(size, bits)
            nbuf = max(2, math.ceil(768 * MiB / (2 * size)))
            src = torch.from_numpy(payload).cuda()
            ins = [src.clone() for _ in range(nbuf)]
            outs = [torch.empty_like(src) for _ in range(nbuf)]
            for variant in (1, 2, 3):
                best, rule = None, None
                rule_kw = rule_shape(A, bits, size, variant, cus)
                for kw in [dict(rule_kw)] + list(candidates(variant, args.quick)):
                    is_rule = rule is None
                    grid = kw.pop("grid")
                    cfg = A.launch_cfg(grid=grid * cus, **kw)
                    A.aes_ctr_crypt(sched, nonce, 1, ins[0], outs[0], cfg=cfg)
                    torch.cuda.synchronize()
                    digest = hashlib.sha256(outs[0].cpu().numpy().tobytes()).hexdigest()
                    if digest != gold[f"{bits}/{size}"]:
                        raise SystemExit(f"candidate {kw} is not bit-exact at AES-{bits} {size} B")
                    ms = time_shape(torch, A, sched, nonce, ins, outs, cfg, size)
                    kw["grid"] = grid
                    tried.append({"key_bits": bits, "size": size, **kw, "us": round(ms * 1e3, 3), "rule": is_rule})
                    if is_rule:
                        rule = (ms, kw)
                    if best is None or ms < best[0]:
                        best = (ms, kw)
                # The rule's shape is timed again last (the first timing of a
                # size can catch clocks still ramping) and keeps the faster of
                # its two; it stays unless a candidate beats it by 1% or more
                # (closer than that is within run-to-run noise).
                rule_cfg = A.launch_cfg(**{k: (v * cus if k == "grid" else v) for k, v in rule[1].items()})
                again = time_shape(torch, A, sched, nonce, ins, outs, rule_cfg, size)
                if again < rule[0]:
                    rule = (again, rule[1])
                    if again < best[0]:
                        best = rule
                chosen = best if best[0] < 0.99 * rule[0] else rule
                ms, kw = chosen
                entry = {"variant": variant, "key_bits": bits, "size_log2": int(math.log2(size)),
                         "bpl": kw.get("blocks_per_lane", 1), "wg": kw["wg_size"],
                         "grid_per_cu": kw["grid"],
                         "copies": kw.get("lds_copies", 0), "tables": kw.get("lds_tables", 0)}
                if variant == 1:
                    entry["first"] = {1: 1, 2: 2, 3: 0}[kw["wave_groups"]]
                entries.append(entry)
                report.append({**entry, "us": round(ms * 1e3, 3), "gbps": round(size / ms / 1e6, 1),
                               "rule_us": round(rule[0] * 1e3, 3), "best_us": round(best[0] * 1e3, 3),
                               "from_rule": chosen is rule})
                print(json.dumps(report[-1]), flush=True)
            del ins, outs, src
            torch.cuda.empty_cache()
    batch_tried = []
    if not args.no_batch:
        entry, batch_tried = tune_batch(torch, A, W, cus, golden["batch_keystream_samples"]["sha256"])
        entries.append(entry)
    with open(args.out, "w") as f:
        json.dump({"generated": time.strftime("%Y-%m-%d %H:%M:%S"), "device": torch.cuda.get_device_name(0),
                   "entries": entries, "measured": report}, f, indent=1)
        f.write("\n")
    print(f"wrote {args.out}")
    if args.report:
        with open(args.report, "w") as f:
            json.dump({"single": tried, "batch": batch_tried, "winners": report}, f, indent=1)
            f.write("\n")


def sampled_keystream_digest(torch, reqs, offs, dst) -> str:
    """SHA-256 over the sampled blocks of every request (blocks 0, n//2 and
    n-1, each once, the last cut to the tail), in request order, read from
    the outputs of a batch run on zero payloads."""
    idx = []
    for r, o in zip(reqs, offs):
        nb = (r.length + 15) // 16
        for j in sorted({0, nb // 2, nb - 1}):
            n = min(16, r.length - 16 * j)
            idx.extend(range(o + 16 * j, o + 16 * j + n))
    sel = dst[torch.tensor(idx, dtype=torch.int64, device=dst.device)]
    return hashlib.sha256(sel.cpu().numpy().tobytes()).hexdigest()


def tune_batch(torch, A, W, cus, expect: str):
    """Tile sizing (tiles per CU and the largest tile) and blocks per lane of
    the batch kernel on the 4096-request batch, on zero payloads: every
    candidate's sampled keystream must hash to `expect`."""
    reqs = W.batch_requests()
    offs, pos = [], 0
    for r in reqs:
        offs.append(pos)
        pos += (r.length + 255) // 256 * 256
    src = torch.zeros(pos, dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    scheds = [A.aes_expand_key(r.key) for r in reqs]
    objs = [A.Request(s, r.nonce, r.ctr0, src.data_ptr() + o, dst.data_ptr() + o, r.length)
            for s, r, o in zip(scheds, reqs, offs)]
    arr = A.make_desc_array(objs)
    total = sum(r.length for r in reqs)
    best, rule, tried = None, None, []
    # The sizing rule's tiles-per-CU constant only matters for batches too
    # small to reach the largest tile, which this workload is not (4.2 GB
    # over 16 tiles per CU would be 1 MiB tiles): it stays at 16, and the
    # largest tile and the blocks per lane are searched, the rule's own
    # (64 KiB, 2) first.
    tpc = 16
    for _ in range(3):          # warm-up: staging, graphs and clocks
        A.aes_ctr_crypt_batch(objs, cfg=A.batch_cfg(tile_bytes=65536, blocks_per_lane=2), descs=arr)
    torch.cuda.synchronize()
    for max_tile, bpl in [(65536, 2)] + list(itertools.product((16384, 32768, 65536, 131072, 262144), (1, 2))):
        if rule is not None and (max_tile, bpl) == (65536, 2):
            continue
        tile = max(2048, min(max_tile, (total // (tpc * cus) + 2047) // 2048 * 2048))
        cfg = A.batch_cfg(tile_bytes=tile, blocks_per_lane=bpl)
        dst.zero_()
        A.aes_ctr_crypt_batch(objs, cfg=cfg, descs=arr)
        torch.cuda.synchronize()
        got = sampled_keystream_digest(torch, reqs, offs, dst)
        if got != expect:
            raise SystemExit(f"batch candidate tiles/CU={tpc} max tile={max_tile} bpl={bpl} is not bit-exact")
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            A.aes_ctr_crypt_batch(objs, cfg=cfg, descs=arr)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = sorted(times)[2]
        rec = {"tiles_per_cu": tpc, "max_tile_bytes": max_tile, "tile_bytes": tile, "bpl": bpl, "ms": round(ms, 3),
               "rule": rule is None}
        tried.append(rec)
        print(json.dumps({"batch": rec}), flush=True)
        if rule is None:
            rule = (ms, tpc, max_tile, bpl)
        if best is None or ms < best[0]:
            best = (ms, tpc, max_tile, bpl)
    del src, dst
    torch.cuda.empty_cache()
    chosen = best if best[0] < 0.99 * rule[0] else rule
    return ({"variant": 10, "key_bits": 0, "size_log2": 0, "bpl": chosen[3], "wg": 1024, "grid_per_cu": 1,
             "copies": 0, "tiles_per_cu": chosen[1], "max_tile_bytes": chosen[2]}, tried)


if __name__ == "__main__":
    main()
