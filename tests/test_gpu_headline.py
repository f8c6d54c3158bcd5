"""Every output of the two full-size batched workloads against the oracle (needs an
MI355X).

* the batched workload: 4,096 queries over a pool of 10,000 bitmaps of 2^22 rows (d
  log-uniform in [1e-4, 0.3], N uniform in [2, 256], T uniform in [1, N]);
* the 10,000 held-out queries of the selector workload, drawn the same way from the
  same pool with their own seed.

Both run in the benchmark's launch: the learned selector's per-query variants, the
tuned grid, graph replays with eager work between them.  The expected results are
stored as the length and SHA-256 digest of the oracle's canonical output of every
query (tests/golden/batched_digests.json, written by make_batched_digests.py, which
calls only the oracle and the generators).  A mismatch recomputes that query with the
oracle and reports the first differing word.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DIGESTS = os.path.join(HERE, "golden", "batched_digests.json")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def env():
    from tests import gpu_util
    E = gpu_util.lib()
    with open(DIGESTS) as f:
        dg = json.load(f)
    n_bits, n_pool = dg["n_bits"], dg["pool"]
    pool, _ = D.config4_pool(n_pool, n_bits)
    bms = E.register_many(pool, n_bits)
    nw = np.array([len(s) for s in pool], dtype=np.int64)
    yield E, dg, pool, bms, nw, n_bits
    for b in bms:
        b.release()


def _check_all(E, name, dg, pool, bms, nw, n_bits, queries, signature):
    import torch
    from paper_1402_4466_amd import selector as S
    from paper_1402_4466_amd.workload import PooledBatch
    want = dg[name]
    assert want["queries"] == len(queries)
    sel = S.load_selector()
    pb = PooledBatch(bms, nw, queries, n_bits, selector=sel, signature=signature)
    _say(f"{name}: {len(queries)} queries, selector {pb.sel_kind}, grid {pb.grid}, "
         f"{pb.input_bytes / 1e9:.1f} GB of input")
    try:
        for rep in range(2):
            pb.out.fill_(-1)
            pb.run()
            torch.cuda.synchronize()
            x = torch.ones(4096, device="cuda").sum()   # eager work between the replays
            torch.cuda.synchronize()
            assert E.device_errors() == 0
            ns, dig = pb.digests()
            bad = [i for i in range(len(queries))
                   if int(ns[i]) != want["words"][i] or dig[i] != want["sha256_16"][i]]
            _say(f"{name} replay {rep}: {len(queries) - len(bad)}/{len(queries)} outputs equal the oracle's")
            for i in bad[:3]:
                q = queries[i]
                ref, _ = O.threshold([pool[j] for j in q.idx], n_bits, q.T, want_hist=False)
                got = pb.result(i)
                k = next((j for j in range(min(len(got), len(ref))) if got[j] != ref[j]), min(len(got), len(ref)))
                _say(f"  query {i} (N={len(q.idx)}, T={q.T}): {len(got)} words vs {len(ref)}; first difference "
                     f"at word {k}")
            assert not bad, f"{len(bad)} of {len(queries)} outputs differ from the oracle (first: {bad[:10]})"
    finally:
        pb.free()
        if hasattr(sel, "free"):
            sel.free()


def test_batched_workload_every_output(env):
    E, dg, pool, bms, nw, n_bits = env
    qs = D.queries(D.SEED_BASE + 4, 4096, dg["pool"], 2, 256)
    _check_all(E, "c4", dg, pool, bms, nw, n_bits, qs, f"c4_q{len(qs)}_pool{dg['pool']}")


def test_heldout_selector_workload_every_output(env):
    E, dg, pool, bms, nw, n_bits = env
    te = D.config5_queries(dg["pool"], 0, 10_000)[1]
    _check_all(E, "c5_heldout", dg, pool, bms, nw, n_bits, te, f"c5_heldout_q{len(te)}_pool{dg['pool']}")
