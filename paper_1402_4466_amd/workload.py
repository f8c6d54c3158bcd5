"""Planned batches over a registered pool: every query's output buffer at its bound
inside one device tensor, one persistent graph-captured launch for all queries,
the kernel variant of each query from a selector (chosen once per plan: a batch's
features do not change), the persistent grid from the autotuner cache."""
from __future__ import annotations

import hashlib

import numpy as np

from . import ewahthr as E


def digest(words: np.ndarray) -> str:
    """First 16 hex digits of the SHA-256 of the little-endian words (the stored digests of the
    batched workloads use the same definition)."""
    return hashlib.sha256(np.asarray(words, dtype="<u8").tobytes()).hexdigest()[:16]


class PooledBatch:
    def __init__(self, bms, nw, queries, n_bits: int, selector=None, signature: str | None = None,
                 grid: int | None = None, use_graph: bool = True, stream=None):
        import torch
        from . import autotune as A
        self.queries = queries
        self.n_bits = n_bits
        nw = np.asarray(nw, dtype=np.int64)
        self.in_words = np.array([int(nw[q.idx].sum()) for q in queries], dtype=np.int64)
        self.caps = [E.output_bound(n_bits, int(w)) for w in self.in_words]
        self.offs = np.concatenate([[0], np.cumsum(self.caps)]).astype(np.int64)
        self.out = torch.zeros(int(self.offs[-1]), dtype=torch.int64, device="cuda")
        self.out_n = torch.zeros(len(queries), dtype=torch.int64, device="cuda")
        base, nbase = self.out.data_ptr(), self.out_n.data_ptr()
        self.batch = E.Batch(bms, [(q.idx, q.T) for q in queries], [base + 8 * int(o) for o in self.offs[:-1]],
                             self.caps, [nbase + 8 * i for i in range(len(queries))], grid=E.num_cus(),
                             use_graph=use_graph)
        self.sel_kind = selector.apply(self.batch, stream) if selector is not None else "default"
        self.tuned = None
        if grid is None:
            self.tuned = A.lookup(f"{signature}_{self.sel_kind}") if signature else None
            grid = int(self.tuned["grid"]) if self.tuned else 2 * E.num_cus()
        self.batch.set_grid(grid)
        if self.tuned:
            self.batch.set_win_batch(int(self.tuned.get("win_batch", 6)))
        self.grid = grid
        self.signature = signature

    @property
    def input_bytes(self) -> int:
        return int(self.in_words.sum()) * 8

    def run(self, stream=None):
        self.batch.run(stream)

    def outputs(self):
        """(lengths, host copy of the packed output words); waits for the device."""
        import torch
        torch.cuda.synchronize()
        ns = self.out_n.cpu().numpy().astype(np.int64)
        host = self.out.cpu().numpy().view(np.uint64)
        return ns, host

    def result(self, i: int, ns=None, host=None) -> np.ndarray:
        if ns is None:
            ns, host = self.outputs()
        return host[self.offs[i]:self.offs[i] + ns[i]]

    def digests(self):
        ns, host = self.outputs()
        return ns, [digest(host[self.offs[i]:self.offs[i] + ns[i]]) for i in range(len(self.queries))]

    def free(self):
        self.batch.free()
