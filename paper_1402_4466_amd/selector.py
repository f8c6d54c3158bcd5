"""Per-query kernel-variant selection for the batched path.

Every variant ("arm") computes the same canonical result; they differ in how
the tile routine spends its work: dense carry-save rows or sparse ripple adds
for whole-tile dirty runs, a binary or a unary per-row counter, how long a
segment may be before it is split across a wavefront, and when the per-group
count bounds are worth counting.  The selector itself lives in the library
(ewah_selector_*): a learned cost model (FP32 MLP trained by the library's own
HIP kernels on timings the batched launch measures) and the paper-style rule set
(least-squares running-time models of the forms of Section 8.1, smallest
estimate taken as in hybrid H, Section 8.2).  This module names the arms,
keeps the numpy definition of the features for tests, and wraps the three ways
of choosing:

  MLPSelector   learned cost model, features -> prediction -> argmin on the device;
  RuleSelector  the rule set of the same model file, on the device;
  FixedSelector one arm for every query.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "selector_model.json")

N_FEATURES = 16

# Arms: (name, dense, walk, litwalk, looped, gate).  All compute identical outputs.
#   sparse_*  bit-sliced binary counter, every dirty word added by ripple carry
#             (the accumulator of BSTM, Section 5.3.1);
#   hybrid_*  the same, with inputs whose dirty run covers a whole tile summed by
#             a carry-save-adder tree (a sideways-sum circuit);
#   looped_*  unary saturating counter with levels 1..T (the Looped recurrence,
#             Section 6.2); taken when T <= bit length of N, else as sparse_*;
#   *_gate*   the per-group count bounds (RBMrg's second case, Section 6.4, inside a
#             tile) counted always, never, or above 1.5x the mean bound instead of
#             above 1.1x (also combined with the long walks, the all-cooperative
#             decode and the unary counter).
ARMS = [
    ("hybrid_w8", True, 8, 8, False, 0),
    ("sparse_w8", False, 8, 8, False, 0),
    ("hybrid_coop", True, 0, 0, False, 0),
    ("sparse_walk64", False, 64, 64, False, 0),
    ("hybrid_walk32", True, 32, 64, False, 0),
    ("hybrid_walk128", True, 128, 255, False, 0),
    ("looped_w8", False, 8, 8, True, 0),
    ("looped_coop", False, 0, 0, True, 0),
    ("hybrid_w8_gate_always", True, 8, 8, False, 1),
    ("hybrid_w8_gate_never", True, 8, 8, False, 2),
    ("hybrid_w8_gate_1.5", True, 8, 8, False, 3),
    ("hybrid_walk128_gate_always", True, 128, 255, False, 1),
    ("sparse_walk64_gate_always", False, 64, 64, False, 1),
    ("hybrid_coop_gate_always", True, 0, 0, False, 1),
    ("looped_coop_gate_1.5", False, 0, 0, True, 3),
    ("hybrid_coop_gate_1.5", True, 0, 0, False, 3),
]


def arm_codes(arms=None):
    from . import ewahthr as E
    return [E.variant_code(d, w, l, looped=lp, gate=g) for (_, d, w, l, lp, g) in (arms or ARMS)]


def features_host(queries, stats, n_bits: int) -> np.ndarray:
    """Reference definition of the 16 features in numpy (the device kernel computes
    the same in FP32; used by tests)."""
    nw = np.array([s["n_words"] for s in stats], dtype=np.float64)
    lit = np.array([s["n_literals"] for s in stats], dtype=np.float64)
    pop = np.array([s["popcount"] for s in stats], dtype=np.float64)
    runs = np.array([s["run_count"] for s in stats], dtype=np.float64)
    r = float(max(n_bits, 1))
    dens = np.maximum(pop / r, 1e-9)
    ld = np.log2(dens)
    out = np.zeros((len(queries), N_FEATURES), dtype=np.float64)
    for i, q in enumerate(queries):
        idx = np.asarray(q[0], dtype=np.int64)
        T = float(q[1])
        N = float(len(idx))
        d = ld[idx]
        w = nw[idx]
        ru = runs[idx]
        out[i] = [
            np.log2(N), np.log2(max(T, 1.0)), T / N, np.log2(N - min(T, N) + 1.0),
            d.mean(), d.max(), d.min(), np.sqrt(max((d * d).mean() - d.mean() ** 2, 0.0)),
            np.log2(ru.sum() + 1.0), np.log2(ru.max() + 1.0),
            np.log2(w.sum() + 1.0), np.log2(w.max() + 1.0),
            lit[idx].sum() / max(w.sum(), 1.0), np.log2(r),
            dens[idx].sum() / max(T, 1.0), 1.0,
        ]
    return out


def rule_regressors(feat: np.ndarray) -> np.ndarray:
    """Regressors of the paper-style running-time model, from the features (numpy
    statement of the library's definition, for tests)."""
    ewah = 2.0 ** feat[:, 10] - 1.0            # total compressed words (EWAHSize / 8)
    N = 2.0 ** feat[:, 0]
    T = 2.0 ** feat[:, 1]
    tiles = np.maximum(2.0 ** feat[:, 13] / 65536.0, 1.0)
    lit = feat[:, 12] * ewah
    return np.stack([ewah, ewah * np.log(np.maximum(N, 1.0)), N * tiles, T * ewah, lit], axis=1)


class FixedSelector:
    kind = "fixed"

    def __init__(self, variant: int = 0):
        self.variant = variant

    def apply(self, batch, stream=None):
        batch.set_variants(np.full(batch.nq, self.variant, dtype=np.uint32))
        return f"fixed:{self.variant:#x}"


class _LibSelector:
    mode = 0
    kind = ""

    def __init__(self, lib_selector):
        self.sel = lib_selector
        self.codes = [int(c) for c in lib_selector.arm_codes()]

    def apply(self, batch, stream=None):
        """Features -> prediction -> argmin, on the device; the choice lands in the batch's
        query records (one call per plan: a batch's features do not change)."""
        batch.select_model(self.sel, self.mode, stream)
        return self.kind

    def free(self):
        self.sel.free()


class MLPSelector(_LibSelector):
    mode = 0
    kind = "mlp"


class RuleSelector(_LibSelector):
    mode = 1
    kind = "rules"


def load_selector(path: str | None = None, kind: str = "mlp"):
    """The library selector of a model file (default: the committed model), or the default
    variant for every query when there is no model file."""
    from . import ewahthr as E
    p = path or DEFAULT_MODEL
    if not os.path.exists(p):
        return FixedSelector(0)
    with open(p) as f:
        m = json.load(f)
    if m.get("kind", "mlp") == "fixed":
        return FixedSelector(int(m.get("variant", 0)))
    sel = E.Selector.load(p)
    return RuleSelector(sel) if kind == "rules" else MLPSelector(sel)
