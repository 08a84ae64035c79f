"""Launch-shape autotuner for the generation kernel.

The lanes given to one individual (`tpr`: 64, 128, 256, 512 or 1024) trade the
number of rows in flight against per-row work; the library's default follows
D and N.  tune_tpr() times every candidate on a scratch handle of the same
shape (results never depend on tpr) and keeps the fastest per device and run
shape in a small JSON cache next to this file."""
from __future__ import annotations

import json
import os

CANDIDATES = (64, 128, 256, 512, 1024)
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")
SHAPE_KEYS = ("dtype", "fn", "xo", "exp_impl", "mm", "N", "D")


def _key(cfg: dict) -> str:
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    return "|".join([dev] + [str(cfg.get(k, "")) for k in SHAPE_KEYS])


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def measure(cfg: dict, tpr: int, gens: int = 64, warmup: int = 4) -> float:
    """Milliseconds per generation of `cfg` with the given lanes per row."""
    import torch

    from . import DE
    gpu = DE([dict(cfg, tpr=tpr)])
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
    if use_cache and key in cache:
        rec = cache[key]
        return int(rec["tpr"]), {int(k): v for k, v in rec["ms"].items()}
    table = {t: measure(cfg, t, gens) for t in candidates}
    best = min(table, key=table.get)
    cache[key] = {"tpr": best, "ms": {str(k): v for k, v in table.items()}}
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, CACHE)
    return best, table
