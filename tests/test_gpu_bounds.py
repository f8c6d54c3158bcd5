"""Per-group count bounds and the batched work split (needs an MI355X).

* Queries just below and above the input count where the tiles switch from
  single-word bounds to 4-word-group bounds (256 / 257 inputs), over bitmaps of
  long runs far apart and with thresholds around the mean bound, so that tiles
  are settled whole, partly pruned or fully decoded.  Plain and batched paths
  are compared word for word with the oracle.
* Batches with fewer (query, tile) items than XCD ranges, and grids of one and
  three workgroups, so that ranges are empty and every item is taken from
  another range.
* Every batch with the bounds pre-pass and without it.
"""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TW = int(re.search(r"#define EWT_TILE_WORDS (\d+)",
                   open(os.path.join(ROOT, "paper_1402_4466_amd", "csrc", "thr_device.h")).read()).group(1))
TW_ROWS = TW * 64   # rows per tile


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def _run_batch(E, G, bms, pool, n_bits, queries, grid=0, use_graph=True, prepass=None):
    import torch
    outs, ns, caps = [], [], []
    for idx, _ in queries:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in idx)))
        outs.append(o); ns.append(n); caps.append(c)
    batch = E.Batch(bms, queries, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns],
                    grid=grid, use_graph=use_graph)
    if prepass is not None:
        batch.set_prepass(prepass)
    batch.run()
    torch.cuda.synchronize()
    got = [G.fetch(outs[i], ns[i]) for i in range(len(queries))]
    batch.free()
    return got


def test_bounds_around_granularity_switch(G):
    E = G.lib()
    n_bits = 5 * TW_ROWS + 777                     # several tiles and a ragged tail
    n = 300
    # runs of ones (mean 400 rows) far apart (mean 4000 rows): inputs overlap in some
    # words and not in others, so word bounds range from a few to ~45 at N ~ 256
    pool = D.bitmaps(D.MARKOV, 400.0, np.full(n, 4000.0), n_bits, [D.key(4242, k) for k in range(n)])
    bms = G.register(pool, n_bits)
    try:
        rng = np.random.default_rng(11)
        queries = []
        for N in (255, 256, 257, 300):
            idx = np.sort(rng.choice(n, N, replace=False)).astype(np.uint32)
            # no word pruned, ~10 % pruned, ~85 % pruned (both with ones in the output), all pruned
            for T in (N // 40, N // 12, N // 8, N // 5):
                queries.append((idx, int(T)))
        wants = [O.threshold([pool[i] for i in idx], n_bits, T, want_hist=False)[0] for idx, T in queries]
        for (idx, T), want in zip(queries, wants):
            got = G.gpu_threshold([bms[i] for i in idx], T)
            assert np.array_equal(got, want), (len(idx), T)
        for pre in (False, True):
            got = _run_batch(E, G, bms, pool, n_bits, queries, prepass=pre)
            for i, want in enumerate(wants):
                assert np.array_equal(got[i], want), ("batched", pre, len(queries[i][0]), queries[i][1])
    finally:
        for b in bms:
            b.release()
    assert E.device_errors() == 0


def test_small_batches_and_grids(G):
    E = G.lib()
    n = 12
    for n_bits, nq in ((TW_ROWS - 5, 1), (TW_ROWS, 3), (TW_ROWS + 1, 1), (2 * TW_ROWS + 9, 3), (TW_ROWS // 3, 7),
                       (TW_ROWS, 8), (TW_ROWS, 9)):
        dens = np.linspace(0.001, 0.3, n)
        pool = D.bitmaps(D.IID, dens, 0.0, n_bits, [D.key(5151 + n_bits % 97, k) for k in range(n)])
        bms = G.register(pool, n_bits)
        try:
            qs = D.queries(606 + nq, nq, n, 1, n)
            queries = [(q.idx, q.T) for q in qs]
            wants = [O.threshold([pool[i] for i in idx], n_bits, T, want_hist=False)[0] for idx, T in queries]
            for grid, pre in [(g, p) for g in (0, 1, 3) for p in (False, True)]:
                got = _run_batch(E, G, bms, pool, n_bits, queries, grid=grid, use_graph=(grid != 3), prepass=pre)
                for i, want in enumerate(wants):
                    assert np.array_equal(got[i], want), (n_bits, nq, grid, pre, i)
        finally:
            for b in bms:
                b.release()
    assert E.device_errors() == 0
