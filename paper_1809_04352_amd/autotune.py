"""Autotuner of the launch configuration of eses_classify.

Times eses_classify for a set of candidate configurations (tile edge and,
for batches, persistent workgroups per compute unit and the order in which
the fused launch takes its units) on the caller's molecules and keeps the
fastest; results are cached per workload signature
(molecule count, atom count and spacing buckets) in a JSON file
($ESES_AUTOTUNE_CACHE, default ~/.cache/eses_autotune.json).  Labels do not
depend on the choice.
"""
from __future__ import annotations

import json
import math
import os

from . import eses

CANDIDATES_SINGLE = [dict(tile=8), dict(tile=4)]
CANDIDATES_BATCH = [dict(tile=8, blocks_per_cu=0, unit_order=0),
                    dict(tile=8, blocks_per_cu=0, unit_order=1),
                    dict(tile=8, blocks_per_cu=5, unit_order=0),
                    dict(tile=4, blocks_per_cu=0, unit_order=0)]


def _cache_path():
    return os.environ.get("ESES_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "eses_autotune.json"))


def signature(mols, prec) -> str:
    n = len(mols)
    atoms = sum(int(m.n_atoms) for m in mols)
    h = min(float(m.spacing) for m in mols)
    return f"n{n}_a{int(math.log2(max(atoms, 1)))}_h{h:.3f}_p{int(prec)}"


def _time_config(mols, prec, cfg, reps, stream):
    import torch
    dims = [eses.grid_dims(m) for m in mols]
    labels = [torch.empty(d[0] * d[1] * d[2], dtype=torch.uint8, device="cuda") for d in dims]
    cand = eses.build_candidates(mols, tile=cfg.get("tile", 0),
                                 blocks_per_cu=cfg.get("blocks_per_cu", 0),
                                 unit_order=cfg.get("unit_order", 0))
    try:
        eses.classify(cand, prec, labels)  # warm-up (records the batch graph)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(reps):
            a.record(stream)
            eses.classify(cand, prec, labels)
            b.record(stream)
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        return best
    finally:
        cand.close()


def tune(mols, prec=eses.ESES_FP32_RECHECK, reps: int = 3, use_cache: bool = True):
    """Returns (config dict, {config: ms}) for the molecules given."""
    import torch
    key = signature(mols, prec)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]["best"], cache[key]["times"]
    stream = torch.cuda.current_stream()
    cands = CANDIDATES_BATCH if len(mols) > 1 else CANDIDATES_SINGLE
    times = {}
    for cfg in cands:
        times[json.dumps(cfg, sort_keys=True)] = _time_config(mols, prec, cfg, reps, stream)
    best = json.loads(min(times, key=times.get))
    if use_cache:
        cache[key] = {"best": best, "times": times}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, times
