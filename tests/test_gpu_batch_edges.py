"""Batched path at the edges of the threshold's range and of the planner's limits (needs an
MI355X).

* T = 0 (every row), T = N + 1 and larger (no row) and N = 1 (the input itself) inside a
  batch whose other queries do real work, on every counter variant and every build of
  the persistent kernel (4..7 windows per wavefront batch), against the oracle;
* the planner sums (query, tile) items in 64 bits and rejects a batch of 2^31 or more
  items before it allocates anything (a 32-bit sum would wrap and size the tile states
  too small).
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D
from tests.ewah_test_util import marker

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def test_batched_trivial_thresholds_and_single_inputs(G):
    import torch
    E = G.lib()
    n_bits = 2 * 512 * 64 + 321            # two full tiles and a ragged one
    pool_n = 24
    d = D.pool_densities(pool_n, seed=4242)
    pool = D.bitmaps(D.IID, d, 0.0, n_bits, [D.key(4242, k) for k in range(pool_n)])
    bms = E.register_many(pool, n_bits)
    rng = np.random.default_rng(4242)
    qs = []
    for i in range(48):
        n = 1 if i % 4 == 0 else int(rng.integers(2, 12))
        idx = rng.choice(pool_n, size=n, replace=False).astype(np.uint32)
        kind = i % 6
        T = {0: 0, 1: n + 1, 2: n + 7, 3: 1, 4: n, 5: int(rng.integers(1, n + 1))}[kind]
        qs.append((idx, T))
    codes = [0, E.variant_code(False, 0, 0), E.variant_code(True, 255, 255), E.variant_code(False, 8, 8, looped=True)]
    outs, ns, caps = [], [], []
    for idx, _ in qs:
        o, n, c = G.alloc_out(n_bits, int(sum(len(pool[i]) for i in idx)))
        outs.append(o); ns.append(n); caps.append(c)
    wants = [O.threshold([pool[i] for i in idx], n_bits, T, want_hist=False)[0] for idx, T in qs]
    batch = E.Batch(bms, qs, [o.data_ptr() for o in outs], caps, [n.data_ptr() for n in ns], use_graph=True)
    try:
        for v, wb in [(c, w) for c in codes for w in (4, 5, 6, 7)]:
            batch.set_variants(np.full(len(qs), v, dtype=np.uint32))
            batch.set_win_batch(wb)
            for rep in range(2):
                _say(f"batched edges: variant {v:#x}, {wb} windows per batch, replay {rep}")
                for o in outs:
                    o.fill_(-1)
                batch.run()
                torch.cuda.synchronize()
                assert E.device_errors() == 0
                for i, (idx, T) in enumerate(qs):
                    got = G.fetch(outs[i], ns[i])
                    assert np.array_equal(got, wants[i]), (v, rep, i, len(idx), T)
    finally:
        batch.free()
        for b in bms:
            b.release()


def test_batch_plan_rejects_item_overflow(G):
    import torch
    E = G.lib()
    # one all-zero bitmap of 2^30 words: 2^21 tiles per query; 2,048 such queries hold 2^32
    # items, 1,024 already reach 2^31
    U = 1 << 30
    n_bits = U * 64
    bms = E.register_many([np.array([marker(0, U, 0)], dtype=np.uint64)], n_bits)
    cap = E.output_bound(n_bits, 1)
    assert cap == 2
    nq = 2048
    out = torch.zeros(nq * cap, dtype=torch.int64, device="cuda")
    out_n = torch.zeros(nq, dtype=torch.int64, device="cuda")
    try:
        with pytest.raises(E.EwahError) as e:
            E.Batch(bms, [([0], 1)] * nq, [out.data_ptr() + 8 * cap * i for i in range(nq)], [cap] * nq,
                    [out_n.data_ptr() + 8 * i for i in range(nq)], use_graph=False)
        assert e.value.code == E.EINVAL and "too many tiles" in str(e.value), str(e.value)
        assert E.device_errors() == 0
    finally:
        for b in bms:
            b.release()
