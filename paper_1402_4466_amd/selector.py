"""Per-query kernel-variant selection.

Every variant ("arm") computes the same canonical result; they differ in how
the tile routine spends its work (dense carry-save rows or sparse ripple adds
for whole-tile dirty runs; a binary or a unary per-row counter; how long a
segment may be before it is split across a wavefront).  Three selectors share one interface:

  MLPSelector   learned cost model: features computed on the device from the
                registration catalog, FP32 MLP (HIP kernels) predicting the
                log-time of every arm, per-query argmin written straight into
                the batch's device query records;
  RuleSelector  paper-style rules: a running-time model per arm of the form
                c1 * EWAHSize + c2 * EWAHSize * ln N + c3 * N * tiles + c4 * T *
                EWAHSize, fitted by least squares to measured times (the
                fitting procedure of Section 8.1), choosing the smallest
                estimate (hybrid H, Section 8.2);
  FixedSelector one arm for every query.

Exhaustive timing (the oracle selector H_opt of Section 8.2) measures
their regret; it lives in train_selector.py.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "selector_model.json")

N_FEATURES = 16

# Arms: (name, dense, walk, litwalk, looped).  All compute identical outputs.
#   sparse_*  bit-sliced binary counter, every dirty word added by ripple carry
#             (the accumulator of BSTM, Section 5.3.1);
#   hybrid_*  the same, with inputs whose dirty run covers a whole tile summed by
#             a carry-save-adder tree (a sideways-sum circuit);
#   looped_*  unary saturating counter with levels 1..T (the Looped recurrence,
#             Section 6.2); taken when T <= bit length of N, else as sparse_*.
ARMS = [
    ("hybrid_w8", True, 8, 8, False),
    ("sparse_w8", False, 8, 8, False),
    ("hybrid_coop", True, 0, 0, False),
    ("sparse_walk64", False, 64, 64, False),
    ("hybrid_walk32", True, 32, 64, False),
    ("hybrid_walk128", True, 128, 255, False),
    ("looped_w8", False, 8, 8, True),
    ("looped_coop", False, 0, 0, True),
]


def arm_codes():
    from . import ewahthr as E
    return [E.variant_code(d, w, l, looped=lp) for (_, d, w, l, lp) in ARMS]


def features_host(queries, stats, n_bits: int) -> np.ndarray:
    """Reference definition of the 16 features in numpy (the device kernel computes
    the same in FP32; used by tests and the rule set)."""
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
    """Regressors of the paper-style running-time model, from the features."""
    ewah = 2.0 ** feat[:, 10] - 1.0            # total compressed words (EWAHSize / 8)
    N = 2.0 ** feat[:, 0]
    T = 2.0 ** feat[:, 1]
    tiles = np.maximum(2.0 ** feat[:, 13] / 65536.0, 1.0)
    lit = feat[:, 12] * ewah
    return np.stack([ewah, ewah * np.log(np.maximum(N, 1.0)), N * tiles, T * ewah, lit], axis=1)


class FixedSelector:
    kind = "fixed"

    def __init__(self, variant: int = 0, grid: int = 0):
        self.variant = variant
        self.grid = grid

    def choose_host(self, feat):
        return np.full(len(feat), self.variant, dtype=np.uint32)

    def apply(self, batch, pool, queries, n_bits, stream=None):
        batch.set_variants(np.full(len(queries), self.variant, dtype=np.uint32))
        return f"fixed:{self.variant:#x}"


class RuleSelector:
    kind = "rules"

    def __init__(self, coef: np.ndarray, codes, grid: int = 0):
        self.coef = np.asarray(coef, dtype=np.float64)     # [n_regressors, K]
        self.codes = [int(c) for c in codes]
        self.grid = grid

    @staticmethod
    def fit(feat: np.ndarray, times: np.ndarray) -> np.ndarray:
        """Least squares through the origin per arm (Section 8.1): times [n, K] in microseconds."""
        X = rule_regressors(feat)
        coef = np.zeros((X.shape[1], times.shape[1]))
        for k in range(times.shape[1]):
            coef[:, k], *_ = np.linalg.lstsq(X, times[:, k], rcond=None)
        return coef

    def predict(self, feat):
        return rule_regressors(feat) @ self.coef

    def choose_arm(self, feat):
        return np.argmin(self.predict(feat), axis=1)

    def choose_host(self, feat):
        return np.asarray([self.codes[j] for j in self.choose_arm(feat)], dtype=np.uint32)

    def apply(self, batch, pool, queries, n_bits, stream=None):
        import torch
        feat = torch.zeros((len(queries), N_FEATURES), dtype=torch.float32, device="cuda")
        batch.features(feat.data_ptr(), stream)
        batch.set_variants(self.choose_host(feat.cpu().numpy().astype(np.float64)))
        return "rules"


class MLPSelector:
    kind = "mlp"

    def __init__(self, model: dict):
        self.model = model
        self.grid = int(model.get("grid", 0))
        self.codes = [int(c) for c in model["arm_codes"]]
        self._pred = None

    def predictor(self):
        if self._pred is None:
            from .mlp import Predictor
            self._pred = Predictor(self.model)
        return self._pred

    def prepare(self, batch, nq: int):
        """Device buffers for per-step selection on one batch."""
        import torch
        self._batch = batch
        self._nq = nq
        self._feat = torch.zeros((nq, N_FEATURES), dtype=torch.float32, device="cuda")
        self._predbuf = torch.zeros((nq, len(self.codes)), dtype=torch.float32, device="cuda")
        self.predictor()

    def apply_device(self, stream=None):
        """Features -> MLP -> argmin, all on the device and asynchronous; the choice lands in the
        batch's query records, read by the next run of the batch."""
        self._batch.features(self._feat.data_ptr(), stream)
        self._pred.forward(self._feat.data_ptr(), self._nq, self._predbuf.data_ptr(), stream)
        self._batch.select_async(self._predbuf.data_ptr(), stream)

    def apply(self, batch, pool, queries, n_bits, stream=None):
        self.prepare(batch, len(queries))
        batch.set_arm_codes(self.codes)
        self.apply_device(stream)
        return "mlp"

    def choose_device_arms(self, feat_ptr: int, n: int):
        import torch
        pred = torch.zeros((n, len(self.codes)), dtype=torch.float32, device="cuda")
        self.predictor().forward(feat_ptr, n, pred.data_ptr())
        return pred.argmin(dim=1).cpu().numpy()


def load_selector(path: str | None = None):
    p = path or DEFAULT_MODEL
    if os.path.exists(p):
        with open(p) as f:
            m = json.load(f)
        kind = m.get("kind", "mlp")
        if kind == "mlp":
            return MLPSelector(m)
        if kind == "rules":
            return RuleSelector(np.asarray(m["coef"]), m["arm_codes"], m.get("grid", 0))
        if kind == "fixed":
            return FixedSelector(int(m.get("variant", 0)), int(m.get("grid", 0)))
    return FixedSelector(0, 0)
