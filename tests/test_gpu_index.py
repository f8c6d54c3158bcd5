"""Many-Criteria and Similarity(n) workloads over synthetic bitmap indexes on the
GPU path (needs an MI355X), against the oracle (Sections 4 and 7.3).

Thresholds are settled by the empty-answer rule with the oracle's largest row
count.  Every query runs through the batched persistent launch (repeated
bitmaps within a query included) and a sample through the plain path; the
GPU opt-threshold (K = 1) must give the oracle's largest count.  Small tables
cover every shape; the full-size tables are checked on a sample of queries.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd.datagen import index as DI

pytestmark = pytest.mark.gpu

SCALE = {"census_like": 0.05, "tweed_like": 1.0, "weather_like": 0.02}


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def _run_index(G, ix, qs, plain_every=5):
    import torch
    E = G.lib()
    bms = E.register_many(ix.streams, ix.n_bits)
    try:
        settled, wants = [], []
        for q in qs:
            streams = [ix.streams[b] for b in q.idx]
            tmax, _ = O.opt_threshold(streams, ix.n_bits, 1)
            T = q.settle(tmax)
            if T is None:
                continue
            settled.append((q, T, tmax))
            wants.append(O.threshold(streams, ix.n_bits, T, want_hist=False)[0])
        assert settled
        outs, ns, caps = [], [], []
        for q, T, _ in settled:
            o, n, c = G.alloc_out(ix.n_bits, int(sum(len(ix.streams[b]) for b in q.idx)))
            outs.append(o); ns.append(n); caps.append(c)
        batch = E.Batch(bms, [(q.idx, T) for q, T, _ in settled], [o.data_ptr() for o in outs], caps,
                        [n.data_ptr() for n in ns], grid=E.num_cus(), use_graph=True)
        for rep in range(2):
            for o in outs:
                o.zero_()
            batch.run()
            torch.cuda.synchronize()
            assert E.device_errors() == 0
            for i, (q, T, _) in enumerate(settled):
                assert np.array_equal(G.fetch(outs[i], ns[i]), wants[i]), (ix.name, q.kind, i, T, rep)
        batch.free()
        for i in range(0, len(settled), plain_every):
            q, T, tmax = settled[i]
            sub = [bms[b] for b in q.idx]
            assert np.array_equal(G.gpu_threshold(sub, T), wants[i]), (ix.name, q.kind, i, "plain")
            o, n, c = G.alloc_out(ix.n_bits, int(sum(len(ix.streams[b]) for b in q.idx)))
            t_gpu = E.opt_threshold(sub, 1, o.data_ptr(), c, n.data_ptr())
            assert t_gpu == tmax, (ix.name, q.kind, i)
        assert E.device_errors() == 0
        return len(settled)
    finally:
        for b in bms:
            b.release()


@pytest.mark.parametrize("shape", DI.SHAPE_NAMES)
def test_small_tables(G, shape):
    ix = DI.build_index(DI.table(shape, SCALE[shape]))
    idx = {shape: ix}
    qs = DI.many_criteria(idx, 40, seed=301, shapes=(shape,)) + DI.similarity(idx, 40, seed=302, shapes=(shape,))
    n = _run_index(G, ix, qs)
    print(f"{shape} x{SCALE[shape]}: {ix.n_bitmaps} bitmaps, {n} queries", flush=True)


@pytest.mark.parametrize("shape", DI.SHAPE_NAMES)
def test_full_size_tables(G, shape):
    ix = DI.build_index(DI.table(shape))
    idx = {shape: ix}
    qs = DI.many_criteria(idx, 24, seed=311, shapes=(shape,)) + DI.similarity(idx, 24, seed=312, shapes=(shape,))
    n = _run_index(G, ix, qs, plain_every=8)
    print(f"{shape}: {ix.n_bitmaps} bitmaps, {n} queries", flush=True)
