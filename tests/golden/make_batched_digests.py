"""Writes batched_digests.json beside this file: for every query of the batched workload
(4,096 queries over a pool of 10,000 bitmaps of 2^22 rows, d log-uniform in [1e-4, 0.3],
N uniform in [2, 256], T uniform in [1, N]) and of the 10,000 held-out queries of the
selector workload (drawn the same way from the same pool with their own seed), the
length in words and the first 16 hex digits of the SHA-256 of the oracle's canonical
EWAH result (little-endian 64-bit words).

It calls only the oracle (oracle/) and the seeded input generators, on host threads (the
C oracle is reentrant and ctypes releases the interpreter lock during the call).

    python tests/golden/make_batched_digests.py [--threads 8]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1402_4466_amd import datagen as D  # noqa: E402

OUT = os.path.join(HERE, "batched_digests.json")
N_BITS = 1 << 22
POOL = 10_000


def digest(words) -> str:
    return hashlib.sha256(words.astype("<u8").tobytes()).hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t0 = time.perf_counter()
    pool, _ = D.config4_pool(POOL, N_BITS)
    sets = {
        "c4": D.queries(D.SEED_BASE + 4, 4096, POOL, 2, 256),
        "c5_heldout": D.config5_queries(POOL, 0, 10_000)[1],
    }

    def one(q):
        out, _ = O.threshold([pool[i] for i in q.idx], N_BITS, q.T, want_hist=False)
        return int(len(out)), digest(out)

    res = {"n_bits": N_BITS, "pool": POOL, "hash": "sha256 of the little-endian words, first 16 hex digits"}
    with ThreadPoolExecutor(max_workers=args.threads) as ex:
        for name, qs in sets.items():
            rows = []
            for k, r in enumerate(ex.map(one, qs)):
                rows.append(r)
                if (k + 1) % 500 == 0:
                    print(f"{name}: {k + 1}/{len(qs)} ({time.perf_counter() - t0:.0f} s)", flush=True)
            res[name] = {"queries": len(qs), "words": [r[0] for r in rows], "sha256_16": [r[1] for r in rows]}
    with open(OUT, "w") as f:
        json.dump(res, f, separators=(",", ":"))
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
