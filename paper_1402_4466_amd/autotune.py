"""Autotuner of the batched launch: grid search over the persistent grid size
for a planned batch, min of repeats, results cached in JSON keyed by GPU
architecture, HIP runtime version and workload signature."""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")


def device_key() -> str:
    import torch
    prop = torch.cuda.get_device_properties(0)
    arch = getattr(prop, "gcnArchName", "unknown").split(":")[0]
    return f"{arch}|hip{torch.version.hip}|cu{prop.multi_processor_count}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(signature: str, path: str = CACHE):
    return load_cache(path).get(f"{device_key()}|{signature}")


def tune_batch(batch, run_step, signature: str, n_cu: int, reps: int = 3, grids=None, path: str = CACHE,
               log=None) -> dict:
    """run_step() launches one full step on the current stream.  Tries each grid
    size, keeps the fastest (min over reps), stores it in the cache."""
    import torch
    grids = grids or sorted({n_cu // 2, (3 * n_cu) // 4, n_cu, (5 * n_cu) // 4, (3 * n_cu) // 2, 2 * n_cu})
    res = {}
    for g in grids:
        batch.set_grid(g)
        run_step()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record()
            run_step()
            e.record()
            e.synchronize()
            best = min(best, s.elapsed_time(e))
        res[str(g)] = round(best, 4)
        if log:
            log(f"  grid {g}: {best:.3f} ms")
    g_best = int(min(res, key=res.get))
    batch.set_grid(g_best)
    entry = {"grid": g_best, "ms": res}
    cache = load_cache(path)
    cache[f"{device_key()}|{signature}"] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return entry
