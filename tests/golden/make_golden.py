"""Write the stored expected values under tests/golden/ from the CPU oracle.

Only ``oracle`` computes anything here; ``workloads`` supplies the seeded
input bytes.  The digests let a GPU test check a full-size output (up to
256 MiB) bit for bit without re-running the slow oracle on that size.

Usage: python tests/golden/make_golden.py [--threads N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def digest(a) -> str:
    return hashlib.sha256(a.tobytes()).hexdigest()


def batch_samples() -> dict:
    """SHA-256 over sampled keystream blocks of the 4096-request batch
    workload: for each request in order, blocks 0, n//2 and n-1 (each once),
    the last one cut to the message's final partial block.  An encryption of
    zero bytes outputs exactly these keystream bytes, so a tuner can check a
    candidate launch shape on zero payloads without the oracle."""
    import numpy as np
    h = hashlib.sha256()
    for r in W.batch_requests():
        nb = (r.length + 15) // 16
        for j in sorted({0, nb // 2, nb - 1}):
            n = min(16, r.length - 16 * j)
            ks = oracle.ctr(r.key, r.nonce, (r.ctr0 + j) & 0xFFFFFFFF, np.zeros(n, np.uint8))
            h.update(ks.tobytes())
    return {"sha256": h.hexdigest(),
            "blocks": "per request: keystream blocks 0, n//2, n-1 (distinct), the last cut to the tail"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    out = {"generator": "tests/golden/make_golden.py (oracle only)",
           "single_1mib": {}, "sweep": {}}

    s = W.single_1mib()
    c = oracle.ctr(s.key, s.nonce, s.ctr0, s.data, threads=args.threads)
    out["single_1mib"] = {"sha256": digest(c), "head16": c[:16].tobytes().hex(),
                          "tail16": c[-16:].tobytes().hex()}

    for bits in (128, 256):
        key, nonce = W.sweep_key(bits)
        for n in W.SWEEP_SIZES + [W.BIG_SIZE]:
            p = W.sweep_payload(n, bits)
            c = oracle.ctr(key, nonce, 1, p, threads=args.threads)
            out["sweep"][f"{bits}/{n}"] = digest(c)
            print(bits, n, out["sweep"][f"{bits}/{n}"], flush=True)

    out["batch_keystream_samples"] = batch_samples()

    with open(os.path.join(HERE, "ctr_digests.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
