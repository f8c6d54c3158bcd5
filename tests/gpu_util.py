"""Helpers for GPU tests: run the HIP path through the C ABI with torch-owned device buffers."""
from __future__ import annotations

import numpy as np

_inited = False


def lib():
    global _inited
    from paper_1402_4466_amd import ewahthr as E
    if not _inited:
        E.init(0)
        _inited = True
    return E


def alloc_out(n_bits: int, sum_words: int):
    import torch
    E = lib()
    cap = max(E.output_bound(n_bits, sum_words), 1)
    out = torch.zeros(cap, dtype=torch.int64, device="cuda")
    out_n = torch.zeros(1, dtype=torch.int64, device="cuda")
    return out, out_n, cap


def fetch(out, out_n) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    n = int(out_n.cpu().item())
    return out[:n].cpu().numpy().view(np.uint64).copy()


def gpu_threshold(bitmaps, T: int, variant: int = 0, stream=None) -> np.ndarray:
    """bitmaps: registered ewahthr.Bitmap list."""
    E = lib()
    n_bits = bitmaps[0].n_bits
    out, out_n, cap = alloc_out(n_bits, sum(b.n_words for b in bitmaps))
    E.threshold(bitmaps, T, out.data_ptr(), cap, out_n.data_ptr(), stream=stream, variant=variant)
    res = fetch(out, out_n)
    assert E.device_errors() == 0
    return res


def register(streams, n_bits: int):
    return lib().register_many(streams, n_bits)
