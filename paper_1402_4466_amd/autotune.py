"""Autotuner of the batched launch: a search over the launch schedule of a planned
batch -- the persistent grid (workgroups), the windows a wavefront decodes per
batch of loads (the persistent kernel is built for 4..7) and whether the bounds
pre-pass runs -- min of repeated timed launches, results cached in JSON keyed by
GPU architecture, HIP runtime version and workload signature.  Results never
depend on the knobs."""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "autotune_cache.json")
WIN_BATCHES = (4, 5, 6, 7)


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


def apply(batch, entry) -> None:
    """Sets a cached schedule on a planned batch (knobs the entry lacks keep the plan's defaults)."""
    batch.set_grid(int(entry["grid"]))
    batch.set_win_batch(int(entry.get("win_batch", 6)))
    if "prepass" in entry:
        batch.set_prepass(bool(entry["prepass"]))


def _time(run_step, reps):
    import torch
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
    return best


def tune_batch(batch, run_step, signature: str, n_cu: int, reps: int = 3, grids=None, win_batches=WIN_BATCHES,
               path: str = CACHE, log=None, prepass=(False, True)) -> dict:
    """run_step() launches one full step on the current stream.  Tries every (grid,
    windows per batch, pre-pass) triple, keeps the fastest (min over reps), stores it
    in the cache."""
    grids = grids or sorted({n_cu, (3 * n_cu) // 2, 2 * n_cu})
    res = {}
    for pre in prepass:
        batch.set_prepass(pre)
        for wb in win_batches:
            batch.set_win_batch(wb)
            for g in grids:
                batch.set_grid(g)
                ms = _time(run_step, reps)
                res[f"{g}/{wb}/{int(pre)}"] = round(ms, 4)
                if log:
                    log(f"  grid {g}, {wb} windows per batch, pre-pass {'on' if pre else 'off'}: {ms:.3f} ms")
    best = min(res, key=res.get)
    g_best, wb_best, pre_best = (int(x) for x in best.split("/"))
    entry = {"grid": g_best, "win_batch": wb_best, "prepass": pre_best, "ms": res}
    apply(batch, entry)
    cache = load_cache(path)
    cache[f"{device_key()}|{signature}"] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return entry
