"""The allocation-free threshold entry point against ewah_threshold (needs an MI355X).

Two calls in a row, the second on a smaller input (fewer tiles, fewer inputs), each
compared word for word with ewah_threshold on the same inputs and with the oracle; then
the size limit of the static scratch.  The scratch keeps the previous call's tile states,
so the second call also checks that stale states of a larger query are never read.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd import datagen as D

pytestmark = pytest.mark.gpu

TW_ROWS = 512 * 64


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from tests import gpu_util
    gpu_util.lib()
    return gpu_util


def _both(G, bms, T):
    E = G.lib()
    n_bits = bms[0].n_bits
    sw = sum(b.n_words for b in bms)
    o1, n1, cap = G.alloc_out(n_bits, sw)
    o2, n2, _ = G.alloc_out(n_bits, sw)
    o2.fill_(-1)
    E.threshold(bms, T, o1.data_ptr(), cap, n1.data_ptr())
    E.threshold_noalloc(bms, T, o2.data_ptr(), cap, n2.data_ptr())
    a, b = G.fetch(o1, n1), G.fetch(o2, n2)
    assert E.device_errors() == 0
    return a, b


def test_noalloc_matches_threshold_on_two_calls(G):
    E = G.lib()
    cases = [(96, 37 * TW_ROWS + 1234, 951), (11, 3 * TW_ROWS + 77, 952)]   # the second is smaller
    for n, n_bits, seed in cases:
        rng = np.random.default_rng(seed)
        dens = rng.uniform(0.001, 0.2, n)
        streams = D.bitmaps(D.MARKOV, 32.0, 32.0 * (1.0 - dens) / dens, n_bits, [D.key(seed, k) for k in range(n)])
        bms = G.register(streams, n_bits)
        try:
            for T in (0, 1, 2, 3, n // 2, n, n + 1):
                _say(f"noalloc: N={n} n_bits={n_bits} T={T}")
                a, b = _both(G, bms, T)
                assert np.array_equal(a, b), (n, n_bits, T)
                want, _ = O.threshold(streams, n_bits, T, want_hist=False)
                assert np.array_equal(b, want), (n, n_bits, T)
        finally:
            for x in bms:
                x.release()


def test_noalloc_size_limit_and_errors(G):
    import torch
    E = G.lib()
    from tests.ewah_test_util import marker
    U = 4097 * 512   # one tile more than the scratch holds
    bms = G.register([np.array([marker(0, U, 0)], dtype=np.uint64)], U * 64)
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    out_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    try:
        with pytest.raises(E.EwahError) as e:
            E.threshold_noalloc(bms, 1, out.data_ptr(), 4, out_n.data_ptr())
        assert e.value.code == E.EINVAL and "4096" in str(e.value)
        with pytest.raises(E.EwahError) as e:
            E.threshold_noalloc(bms, 1, out.data_ptr(), 1, out_n.data_ptr())
        assert e.value.code == E.ENOSPC
    finally:
        for x in bms:
            x.release()
    small = G.register([np.array([marker(1, 4, 0)], dtype=np.uint64)], 4 * 64)
    try:
        E.threshold_noalloc(small, 1, out.data_ptr(), 4, out_n.data_ptr())
        torch.cuda.synchronize()
        assert int(out_n[0].item()) == 1 and int(out[0].item()) == marker(1, 4, 0)
    finally:
        small[0].release()
