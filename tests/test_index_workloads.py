"""Bitmap-index workloads (Sections 4 and 7.3), CPU only.

* The generated index is a bitmap index of its table: each bitmap, decoded by
  the oracle, holds exactly the rows with its attribute value; the bitmaps of
  one attribute partition the rows; every stream is canonical.
* The oracle's threshold over a Many-Criteria or Similarity query equals the
  query written as in Section 4, evaluated on the table itself: row i is in the
  answer when the number of criteria (attribute j = value v) it meets is at
  least T.  That evaluation never sees a bitmap, so it pins the oracle on these
  workloads.
* Similarity: every prototype meets all d criteria, so it is in the answer at
  any T <= d.
* The query generators follow Section 7.3 (N range, distinct attributes,
  candidate thresholds, prototypes), deterministically.
* The empty-answer rule: the settled threshold is the first candidate with a
  non-empty answer, and each earlier candidate has an empty one.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1402_4466_amd.datagen import index as DI

SCALE = {"census_like": 0.02, "tweed_like": 0.3, "weather_like": 0.005}


@pytest.fixture(scope="module")
def small():
    return {sh: DI.build_index(DI.table(sh, SCALE[sh])) for sh in DI.SHAPE_NAMES}


def _criteria_count(ix, q):
    """Per row, how many of the query's criteria it meets (from the table)."""
    t = ix.table
    c = np.zeros(t.n_rows, dtype=np.int64)
    for b in q.idx:
        c += t.values[ix.attr[b]] == ix.value[b]
    return c


def _rows(stream, n_bits):
    d = O.decode(stream, n_bits)
    bits = np.unpackbits(d.view(np.uint8), bitorder="little")[:n_bits]
    return np.nonzero(bits)[0]


def test_index_is_a_bitmap_index(small):
    for sh, ix in small.items():
        t = ix.table
        assert len(ix.first) == t.n_attrs + 1 and ix.first[-1] == ix.n_bitmaps
        for j in range(t.n_attrs):
            seen = np.zeros(t.n_rows, dtype=np.int64)
            for b in range(ix.first[j], ix.first[j + 1]):
                assert ix.attr[b] == j
                rows = _rows(ix.streams[b], ix.n_bits)
                want = np.nonzero(t.values[j] == ix.value[b])[0]
                assert len(want) > 0 and np.array_equal(rows, want), (sh, j, b)
                assert ix.bitmap_of[j][ix.value[b]] == b
                seen[rows] += 1
                assert np.array_equal(O.encode(O.decode(ix.streams[b], ix.n_bits), ix.n_bits), ix.streams[b])
            assert (seen == 1).all(), (sh, j)


def test_full_size_shapes():
    """Row, attribute and bitmap counts of the full-size tables (Table real-data-char)."""
    want = {"census_like": (199_523, 42, 103_419), "tweed_like": (11_245, 53, 1_167),
            "weather_like": (1_015_367, 19, 18_647)}
    for sh in ("tweed_like", "census_like"):
        t = DI.table(sh)
        r, d, nb = want[sh]
        assert t.n_rows == r and t.n_attrs == d
        present = sum(int((np.bincount(t.values[j], minlength=t.cards[j]) > 0).sum()) for j in range(d))
        assert abs(present - nb) <= 0.03 * nb, (sh, present)


def test_generators_follow_the_workload_rules(small):
    mc = DI.many_criteria(small, 300, seed=77)
    sim = DI.similarity(small, 300, seed=78)
    assert [q.idx.tolist() for q in mc] == [q.idx.tolist() for q in DI.many_criteria(small, 300, seed=77)]
    assert [q.t_chain for q in sim] == [q.t_chain for q in DI.similarity(small, 300, seed=78)]
    for q in mc + sim:
        ix = small[q.shape]
        ch = q.t_chain
        assert ch[0] <= q.n_attrs - 1 and ch[-1] == 2 and all(a > b for a, b in zip(ch, ch[1:])), ch
    for q in mc:
        ix = small[q.shape]
        assert 3 <= len(q.idx) <= 1000
        assert q.n_attrs == len(np.unique(ix.attr[q.idx])) >= 3
    Ns = np.array([len(q.idx) for q in mc])
    # log N uniform in [log 3, log 1000]: P(N < 30) = log(29.5 / 3) / log(1000 / 3) = 0.393
    assert abs((Ns < 30).mean() - 0.393) < 0.08 and Ns.max() > 300
    for q in sim:
        ix = small[q.shape]
        t = ix.table
        assert len(set(q.prototypes.tolist())) == len(q.prototypes) in DI.SIM_PROTOTYPES
        want = sorted({int(ix.bitmap_of[j][t.values[j, p]]) for j in range(t.n_attrs) for p in q.prototypes})
        assert q.idx.tolist() == want and q.n_attrs == t.n_attrs
    assert {q.shape for q in mc} == set(DI.SHAPE_NAMES) == {q.shape for q in sim}


def test_oracle_matches_the_sql_formulation(small):
    """Section 4: the CASE-sum of the criteria at least T, evaluated on the table."""
    qs = DI.many_criteria(small, 40, seed=91) + DI.similarity(small, 40, seed=92)
    for q in qs:
        ix = small[q.shape]
        cnt = _criteria_count(ix, q)
        streams = [ix.streams[b] for b in q.idx]
        for T in sorted({q.t_chain[0], q.t_chain[-1], 1, len(q.idx)}):
            got, _ = O.threshold(streams, ix.n_bits, T, want_hist=False)
            assert np.array_equal(_rows(got, ix.n_bits), np.nonzero(cnt >= T)[0]), (q.kind, q.shape, T)
        if q.kind == "similarity":
            assert (cnt[q.prototypes] == ix.table.n_attrs).all()
            got, _ = O.threshold(streams, ix.n_bits, q.t_chain[0], want_hist=False)
            assert set(q.prototypes.tolist()) <= set(_rows(got, ix.n_bits).tolist())


def test_empty_answer_rule(small):
    """The settled T is the first candidate with a non-empty answer; a query with
    an empty answer at T = 2 is dropped."""
    qs = DI.many_criteria(small, 60, seed=93)
    dropped = 0
    for q in qs:
        ix = small[q.shape]
        streams = [ix.streams[b] for b in q.idx]
        tmax, _ = O.opt_threshold(streams, ix.n_bits, 1)
        assert tmax == _criteria_count(ix, q).max()
        T = q.settle(tmax)
        for c in q.t_chain:
            res, _ = O.threshold(streams, ix.n_bits, c, want_hist=False)
            empty = len(_rows(res, ix.n_bits)) == 0
            if T is not None and c == T:
                assert not empty
                break
            assert empty, (q.t_chain, c, tmax)
        dropped += T is None
    assert dropped < len(qs)
