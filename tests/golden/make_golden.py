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

    with open(os.path.join(HERE, "ctr_digests.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
