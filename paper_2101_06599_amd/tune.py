"""Launch-shape autotuner for the generation kernels.

The lanes given to one individual (`tpr`: 64, 128, 256, 512 or 1024; batched
launches 64, 128 or 256) trade the number of rows in flight against per-row
work; the library's default follows D and N.  tune_tpr() times every
candidate on a scratch handle of the same shape (results never depend on tpr
beyond the rounding order of fitness sums) and keeps the fastest in a small
JSON cache next to this file, keyed by device, dtype, function, crossover and
the power-of-two buckets of D and N, so that one measurement serves nearby
shapes.  tune_batched() does the same for a table of runs stepped together,
and tune_rot_tile() picks the split-bf16 product's tile shape (`tile` 1-3)
for a rotated run.
"""
from __future__ import annotations

import json
import math
import os

CANDIDATES = (64, 128, 256, 512, 1024)
BATCHED = (64, 128, 256)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
SHAPE_KEYS = ("dtype", "fn", "xo", "exp_impl", "mm")


def bucket(v: int) -> int:
    """The power of two at or above v (the D and N buckets of the cache key)."""
    return 1 << max(0, math.ceil(math.log2(max(1, int(v)))))


def _device() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def _key(cfg: dict) -> str:
    return "|".join([_device()] + [str(cfg.get(k, "")) for k in SHAPE_KEYS] +
                    [f"D{bucket(cfg['D'])}", f"N{bucket(cfg['N'])}"])


def _batch_key(cfgs: list) -> str:
    Ds = sorted(bucket(c["D"]) for c in cfgs)
    fns = sorted({str(c.get("fn", "")) for c in cfgs})
    return "|".join([_device(), "batched", str(cfgs[0].get("dtype", "")), ",".join(fns),
                     f"runs{bucket(len(cfgs))}", f"Dmed{Ds[len(Ds) // 2]}"])


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, best: int, table: dict) -> None:
    cache = _load()
    cache[key] = {"best": best, "ms": {str(k): v for k, v in table.items()}}
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, CACHE)


def measure(cfgs, tpr: int, gens: int = 64, warmup: int = 4) -> float:
    """Milliseconds per generation of one run (dict) or a batch (list) with the
    given lanes per row."""
    import torch

    from . import DE
    runs = [cfgs] if isinstance(cfgs, dict) else list(cfgs)
    gpu = DE([dict(c, tpr=tpr) for c in runs])
    try:
        gpu.generation(warmup)
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        gpu.generation(gens)
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / gens
    finally:
        gpu.close()


def tune_tpr(cfg: dict, gens: int = 64, candidates=CANDIDATES, use_cache: bool = True):
    """(fastest tpr, {tpr: ms per generation}) for one run description."""
    key = _key(cfg)
    cache = _load()
    if use_cache and key in cache and "best" in cache[key]:
        rec = cache[key]
        return int(rec["best"]), {int(k): v for k, v in rec["ms"].items()}
    table = {t: measure(cfg, t, gens) for t in candidates}
    best = min(table, key=table.get)
    _store(key, best, table)
    return best, table


def tune_batched(cfgs: list, gens: int = 32, candidates=BATCHED, use_cache: bool = True):
    """(fastest tpr, {tpr: ms per generation}) for a table of runs launched
    together (one width for the whole batch)."""
    key = _batch_key(cfgs)
    cache = _load()
    if use_cache and key in cache and "best" in cache[key]:
        rec = cache[key]
        return int(rec["best"]), {int(k): v for k, v in rec["ms"].items()}
    table = {t: measure(cfgs, t, gens) for t in candidates}
    best = min(table, key=table.get)
    _store(key, best, table)
    return best, table


def _time_gens(cfgs, gens: int, warmup: int = 2) -> float:
    import torch

    from . import DE
    gpu = DE(list(cfgs))
    try:
        gpu.generation(warmup)
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        gpu.generation(gens)
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / gens
    finally:
        gpu.close()


def tune_rot_tile(cfg: dict, gens: int = 10, use_cache: bool = True):
    """(fastest tile, {tile: ms per generation}) for a rotated run in a
    split-bf16 mode (cfg carries its device rotation tensor `rot`)."""
    key = "tile|" + _key(cfg)
    cache = _load()
    if use_cache and key in cache and "best" in cache[key]:
        rec = cache[key]
        return int(rec["best"]), {int(k): v for k, v in rec["ms"].items()}
    table = {t: _time_gens([dict(cfg, tile=t)], gens) for t in (1, 2, 3)}
    best = min(table, key=table.get)
    _store(key, best, table)
    return best, table
