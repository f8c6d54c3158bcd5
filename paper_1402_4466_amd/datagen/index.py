"""Synthetic relational tables, their bitmap indexes, and the Many-Criteria and
Similarity(n) query workloads over them (Sections 4 and 7.3).

Input generation only: nothing here counts criteria, evaluates a threshold or
decodes a stream.  The empty-answer rule of Section 7.3 needs the largest row
count of a query; the caller supplies it (`IndexQuery.settle`).

Tables.  A table has r rows and d attributes; the bitmap index has one bitmap
per attribute value that occurs (the bitmap of value v of attribute j holds
the rows whose attribute j equals v).  The paper's relational datasets are not
available; three shapes stand in for them, with their row and attribute counts
and (approximately) their bitmap counts (Table real-data-char):

  census_like   r = 199,523    d = 42   41 ordinary attributes with 3,619
                values in all, plus one near-unique attribute (135,000
                values drawn uniformly; about 99,600 occur)
  tweed_like    r = 11,245     d = 53   1,167 values in all
  weather_like  r = 1,015,367  d = 19   18,647 values in all

Recipe per table (seed SEED_BASE + 20 + shape number):
  * cardinality of ordinary attribute j: c_j = max(2, round(total * w_j / sum w)),
    w_j log-uniform in [1, W] (a few wide attributes, many narrow ones), W =
    1,000 census_like, 200 tweed_like, 3,000 weather_like: W sets how narrow
    the narrow attributes are, so the mean density of a bitmap that a
    Many-Criteria query picks (1 / cardinality, averaged over attributes)
    comes near the table's (0.15, 0.20, 0.076);
  * values of attribute j: Zipf(1) over its c_j values (P(v) proportional to
    1 / (v + 1)); the near-unique attribute is uniform;
  * row order: row i keeps row i-1's value of attribute j with probability
    rho_j (rho_j uniform in [0, rho_max]; rho_max = 0.2 census_like, 0.5
    tweed_like, 0.95 weather_like), else draws a fresh value; the fresh draws
    of all rows come first, so rho only sets run lengths, not the value law.
    census_like rows are close to iid (the census extract is unsorted), the
    weather_like rows carry long runs (one month of station readings in time
    order).

Random numbers: the counter-based SplitMix64 stream of the generator library
(`uniform`), one stream per (table, attribute, purpose) and per query.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import SEED_BASE, key, lib, uniform

SHAPES = {
    "census_like": dict(no=0, r=199_523, d=42, total=3_619, big=135_000, skew=1_000.0, rho_max=0.2),
    "tweed_like": dict(no=1, r=11_245, d=53, total=1_167, big=0, skew=200.0, rho_max=0.5),
    "weather_like": dict(no=2, r=1_015_367, d=19, total=18_647, big=0, skew=3_000.0, rho_max=0.95),
}
SHAPE_NAMES = ("census_like", "tweed_like", "weather_like")


@dataclass
class Table:
    name: str
    n_rows: int
    values: np.ndarray        # int32 [d, n_rows]: value code of attribute j in row i
    cards: np.ndarray         # int64 [d]: number of possible values per attribute

    @property
    def n_attrs(self) -> int:
        return self.values.shape[0]


@dataclass
class BitmapIndex:
    """One canonical EWAH bitmap per occurring (attribute, value); bitmaps of
    attribute j are first[j] .. first[j+1]-1, in increasing value order."""
    name: str
    n_bits: int
    streams: list             # list[np.ndarray uint64]
    attr: np.ndarray          # int32 [n_bitmaps]
    value: np.ndarray         # int32 [n_bitmaps]
    first: np.ndarray         # int64 [d + 1]
    table: Table
    bitmap_of: list = field(default_factory=list)   # per attribute: value code -> bitmap id (-1 if absent)

    @property
    def n_bitmaps(self) -> int:
        return len(self.streams)

    @property
    def n_words(self) -> np.ndarray:
        return np.array([len(s) for s in self.streams], dtype=np.int64)


def _zipf_cdf(c: int) -> np.ndarray:
    p = 1.0 / np.arange(1, c + 1, dtype=np.float64)
    cdf = np.cumsum(p)
    return cdf / cdf[-1]


def table(shape: str, scale: float = 1.0) -> Table:
    """The table of one shape; scale < 1 shrinks the row count and every
    cardinality by that factor (for tests)."""
    sp = SHAPES[shape]
    seed = SEED_BASE + 20 + sp["no"]
    r = max(1, int(round(sp["r"] * scale)))
    d = sp["d"]
    n_ord = d - (1 if sp["big"] else 0)
    total = max(2 * n_ord, int(round(sp["total"] * scale)))
    uw = uniform(key(seed, 0xC0), n_ord)
    w = np.exp(np.log(sp["skew"]) * uw)
    cards = np.maximum(2, np.round(total * w / w.sum())).astype(np.int64)
    if sp["big"]:
        cards = np.concatenate([cards, [max(2, int(round(sp["big"] * scale)))]])
    rho = sp["rho_max"] * uniform(key(seed, 0xC1), d)
    vals = np.empty((d, r), dtype=np.int32)
    for j in range(d):
        u = uniform(key(seed, 2 * j), r)
        c = int(cards[j])
        if sp["big"] and j == d - 1:
            fresh = np.minimum((u * c).astype(np.int64), c - 1)
        else:
            fresh = np.minimum(np.searchsorted(_zipf_cdf(c), u, side="left"), c - 1)
        stick = uniform(key(seed, 2 * j + 1), r) < rho[j]
        stick[0] = False
        src = np.where(stick, 0, np.arange(r))
        np.maximum.accumulate(src, out=src)
        vals[j] = fresh[src]
    return Table(shape, r, vals, cards)


def build_index(t: Table) -> BitmapIndex:
    """Bitmap index of a table: one bitmap per occurring attribute value."""
    import ctypes
    L = lib()
    if not hasattr(L, "_rows_sig"):
        vp = ctypes.c_void_p
        L.ewahgen_rows_batch.restype = None
        L.ewahgen_rows_batch.argtypes = [ctypes.c_int, vp, vp, ctypes.c_uint64, vp, vp, vp]
        L._rows_sig = True
    r = t.n_rows
    U = (r + 63) // 64
    streams, attrs, values, first, bitmap_of = [], [], [], [0], []
    for j in range(t.n_attrs):
        col = t.values[j]
        c = int(t.cards[j])
        order = np.argsort(col, kind="stable").astype(np.uint32)      # rows grouped by value, ascending
        counts = np.bincount(col, minlength=c)
        present = np.nonzero(counts)[0]
        offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.uint64)
        # the rows of present[k] are order[row_off[k] : row_off[k+1]] (absent values take no room)
        row_off = np.concatenate([offs[present], [offs[-1]]]).astype(np.uint64)
        m = counts[present].astype(np.uint64)
        caps = np.minimum(np.uint64(U + 1), 2 * m + 2)
        out_off = np.concatenate([[0], np.cumsum(caps)]).astype(np.uint64)
        out = np.empty(max(int(out_off[-1]), 1), dtype=np.uint64)
        n_out = np.empty(len(present), dtype=np.uint64)
        L.ewahgen_rows_batch(len(present), row_off.ctypes.data, order.ctypes.data, r, out_off.ctypes.data,
                             out.ctypes.data, n_out.ctypes.data)
        if len(present) and (n_out == np.uint64(2**64 - 1)).any():
            raise RuntimeError("index generator: bad row list or room too small")
        for k in range(len(present)):
            o = int(out_off[k])
            streams.append(out[o:o + int(n_out[k])].copy())
        m_of = np.full(c, -1, dtype=np.int64)
        m_of[present] = first[-1] + np.arange(len(present))
        bitmap_of.append(m_of)
        attrs.append(np.full(len(present), j, dtype=np.int32))
        values.append(present.astype(np.int32))
        first.append(first[-1] + len(present))
    return BitmapIndex(t.name, r, streams, np.concatenate(attrs), np.concatenate(values),
                       np.array(first, dtype=np.int64), t, bitmap_of)


# ------------------------------------------------------------------ queries

SIM_PROTOTYPES = (1, 5, 10, 15, 20)   # Similarity(n), 20 % each


@dataclass
class IndexQuery:
    """Bitmap ids of the criteria (repeats possible for Many-Criteria), the
    number N' of distinct attributes they constrain, and the candidate
    thresholds: t_chain[0] uniform in [2, N'-1], each next one uniform in
    [2, previous - 1], down to 2."""
    kind: str                 # "many_criteria" or "similarity"
    shape: str
    idx: np.ndarray           # uint32 bitmap ids into the index of `shape`
    n_attrs: int
    t_chain: list
    prototypes: np.ndarray | None = None   # Similarity: the prototype rows

    def settle(self, max_count: int):
        """The threshold the workload runs, given the largest row count over
        the query's bitmaps: the first candidate whose answer is non-empty
        (candidate <= max_count); None when even T = 2 gives an empty answer
        (the query is dropped)."""
        for t in self.t_chain:
            if t <= max_count:
                return t
        return None


def _chain(u: np.ndarray, n_attrs: int) -> list:
    t = 2 + min(int(u[0] * (n_attrs - 2)), n_attrs - 3)     # uniform in [2, N'-1]
    out, k = [t], 1
    while t > 2:
        if k == len(u):                                        # out of draws (p < 2^-40): end at 2
            out.append(2)
            break
        t = 2 + min(int(u[k] * (t - 2)), t - 3)               # uniform in [2, t-1]
        out.append(t)
        k += 1
    return out


_CHAIN_DRAWS = 64          # a chain from N' - 1 <= 11,115 halves on average: far below 64 steps


def many_criteria(indexes: dict, n_queries: int, seed: int | None = None, shapes=SHAPE_NAMES) -> list:
    """Many-Criteria queries (Section 7.3): a table shape uniformly, N from the
    discretized log-uniform law (log N uniform in [log 3, log 1000], N the
    nearest integer), N attributes uniformly with replacement, one bitmap of
    each uniformly; a draw with fewer than 3 distinct attributes is drawn
    again (no threshold lies in [2, N'-1])."""
    seed = SEED_BASE + 30 if seed is None else seed
    out = []
    for q in range(n_queries):
        for attempt in range(1000):
            u = uniform(key(seed, q + (attempt << 32)), 2 + 2 * 1000 + _CHAIN_DRAWS)
            shape = shapes[min(int(u[0] * len(shapes)), len(shapes) - 1)]
            ix = indexes[shape]
            d = len(ix.first) - 1
            n = int(round(math.exp(math.log(3) + u[1] * (math.log(1000) - math.log(3)))))
            n = min(max(n, 3), 1000)
            a = np.minimum((u[2:2 + n] * d).astype(np.int64), d - 1)
            nb = ix.first[a + 1] - ix.first[a]
            b = ix.first[a] + np.minimum((u[2 + 1000:2 + 1000 + n] * nb).astype(np.int64), nb - 1)
            n_attrs = len(np.unique(a))
            if n_attrs >= 3:
                out.append(IndexQuery("many_criteria", shape, b.astype(np.uint32), n_attrs,
                                      _chain(u[2 + 2 * 1000:], n_attrs)))
                break
        else:
            raise RuntimeError("many_criteria: no query with three distinct attributes")
    return out


def similarity(indexes: dict, n_queries: int, seed: int | None = None, shapes=SHAPE_NAMES) -> list:
    """Similarity(n) queries (Section 7.3): a table shape uniformly, n from
    {1, 5, 10, 15, 20} with equal probability, n distinct prototype rows
    uniformly, and every bitmap holding at least one prototype (the values the
    prototypes take).  N' = d: every attribute carries a criterion."""
    seed = SEED_BASE + 31 if seed is None else seed
    out = []
    for q in range(n_queries):
        u = uniform(key(seed, q), 2 + 4 * max(SIM_PROTOTYPES) + _CHAIN_DRAWS)
        shape = shapes[min(int(u[0] * len(shapes)), len(shapes) - 1)]
        ix = indexes[shape]
        t = ix.table
        n = SIM_PROTOTYPES[min(int(u[1] * len(SIM_PROTOTYPES)), len(SIM_PROTOTYPES) - 1)]
        n = min(n, t.n_rows)
        protos, k = [], 2
        while len(protos) < n:              # distinct rows by rejection (4n draws are ample for r >> n)
            if k >= 2 + 4 * max(SIM_PROTOTYPES):
                raise RuntimeError("similarity: too few distinct prototype draws")
            row = min(int(u[k] * t.n_rows), t.n_rows - 1)
            k += 1
            if row not in protos:
                protos.append(row)
        protos = np.array(protos, dtype=np.int64)
        ids = []
        for j in range(t.n_attrs):
            for v in np.unique(t.values[j, protos]):
                ids.append(ix.bitmap_of[j][v])
        d = t.n_attrs
        out.append(IndexQuery("similarity", shape, np.array(sorted(ids), dtype=np.uint32), d,
                              _chain(u[2 + 4 * max(SIM_PROTOTYPES):], d), protos))
    return out
