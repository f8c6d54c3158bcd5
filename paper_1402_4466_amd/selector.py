"""Per-query kernel-variant selection.

Features come from the per-bitmap catalog computed at registration (the kind
of statistics the paper's hybrid assumes a database keeps: compressed size,
cardinality, run counts -- Section 8.1).  Three selectors share one interface:

  RuleSelector     paper-style rules (RBMrg case analysis of Section 6.4 and the
                   cost-model comparison of Section 8.2), with constants refit
                   from timings on this GPU;
  MLPSelector      FP32 MLP 16 -> 64 -> 64 -> K predicting log-time of each
                   variant; trained and evaluated by the library's HIP kernels
                   (machine-learned algorithm selection is the paper's stated
                   future work, Section 9);
  FixedSelector    one variant for every query.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "selector_model.json")

N_FEATURES = 16

# Variant arms: (name, dense, walk, litwalk).  Results are identical for all arms.
ARMS = [
    ("hybrid", True, 8, 8),
    ("sparse", False, 8, 8),
    ("dense_coop", True, 0, 0),
    ("sparse_walk", False, 64, 64),
    ("dense_walk", True, 32, 64),
    ("sparse_coop", False, 0, 0),
]


def arm_codes():
    from . import ewahthr as E
    return [E.variant_code(d, w, l) for (_, d, w, l) in ARMS]


def features(queries, stats, n_bits: int) -> np.ndarray:
    """[Q, 16] float32 features of each query (idx, T) from per-bitmap catalog stats."""
    nw = np.array([s["n_words"] for s in stats], dtype=np.float64)
    lit = np.array([s["n_literals"] for s in stats], dtype=np.float64)
    pop = np.array([s["popcount"] for s in stats], dtype=np.float64)
    runs = np.array([s["run_count"] for s in stats], dtype=np.float64)
    r = float(max(n_bits, 1))
    dens = np.maximum(pop / r, 1e-9)
    ld = np.log2(dens)
    out = np.zeros((len(queries), N_FEATURES), dtype=np.float32)
    for i, q in enumerate(queries):
        idx = np.asarray(q.idx if hasattr(q, "idx") else q[0], dtype=np.int64)
        T = float(q.T if hasattr(q, "T") else q[1])
        N = float(len(idx))
        d = ld[idx]
        w = nw[idx]
        ru = runs[idx]
        out[i] = [
            np.log2(N), np.log2(max(T, 1.0)), T / N, np.log2(N - min(T, N) + 1.0),
            d.mean(), d.max(), d.min(), d.std(),
            np.log2(ru.sum() + 1.0), np.log2(ru.max() + 1.0),
            np.log2(w.sum() + 1.0), np.log2(w.max() + 1.0),
            lit[idx].sum() / max(w.sum(), 1.0), np.log2(r),
            dens[idx].sum() / max(T, 1.0), 1.0,
        ]
    return out


class FixedSelector:
    kind = "fixed"

    def __init__(self, variant: int = 0, grid: int = 0):
        self.variant = variant
        self.grid = grid

    def choose(self, feats, queries):
        return [self.variant] * len(queries), f"fixed:{self.variant:#x}"


class RuleSelector:
    """Paper-style rule set.  Per query: if the inputs are dense enough that most
    tiles are covered by whole-tile dirty runs, use the carry-save-adder arm; if
    they are sparse (few words per tile per input), walk segments with single
    lanes; otherwise the hybrid default.  Thresholds are refit by the tuner."""
    kind = "rules"

    def __init__(self, dense_lit_frac: float = 0.6, walk_words_per_tile: float = 24.0, grid: int = 0):
        self.dense_lit_frac = dense_lit_frac
        self.walk_words_per_tile = walk_words_per_tile
        self.grid = grid

    def choose(self, feats, queries):
        codes = arm_codes()
        out = []
        tiles = np.maximum(2.0 ** feats[:, 13] / 65536.0, 1.0)
        for i in range(len(queries)):
            lit_frac = feats[i, 12]
            words_per_tile_per_input = 2.0 ** feats[i, 10] / tiles[i] / 2.0 ** feats[i, 0]
            if lit_frac >= self.dense_lit_frac:
                out.append(codes[0])
            elif words_per_tile_per_input <= self.walk_words_per_tile:
                out.append(codes[3])
            else:
                out.append(codes[0])
        return out, "rules"


class MLPSelector:
    kind = "mlp"

    def __init__(self, model: dict):
        self.model = model
        self.grid = int(model.get("grid", 0))

    def predict(self, feats):
        from . import mlp
        return mlp.infer(self.model, feats)

    def choose(self, feats, queries):
        codes = [int(c) for c in self.model["arm_codes"]]
        pred = self.predict(feats)
        return [codes[int(j)] for j in np.argmin(pred, axis=1)], "mlp"


def load_selector(path: str | None = None):
    p = path or DEFAULT_MODEL
    if os.path.exists(p):
        with open(p) as f:
            m = json.load(f)
        kind = m.get("kind", "mlp")
        if kind == "mlp":
            return MLPSelector(m)
        if kind == "rules":
            return RuleSelector(m.get("dense_lit_frac", 0.6), m.get("walk_words_per_tile", 24.0), m.get("grid", 0))
        if kind == "fixed":
            return FixedSelector(int(m.get("variant", 0)), int(m.get("grid", 0)))
    return FixedSelector(0, 0)
