"""Autotuner of the launch parameters of tracking calls.

Searches the persistent tracklet kernel's grid size and hipGraph replay on a
given event set and keeps the fastest setting in a JSON cache keyed by the
device name and the workload size bucket.  Results never depend on the
tuning (the tracking output is identical for every setting); only time does.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import torch

from .tracker import Tracker

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")
GRIDS = (0, 512, 768, 1024, 2048)


def _key(n_clusters: int, n_events: int) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    bucket = 1 << max(0, int(math.ceil(math.log2(max(n_clusters, 1)))))
    return f"{dev}|clusters<={bucket}|events={n_events}"


def time_config(trk: Tracker, events: Sequence[tuple], reps: int) -> float:
    batch = len(events) > 1
    run = (lambda: trk.track_batch(events)) if batch else (lambda: trk.track(*events[0]))
    run()                                    # warm-up (and graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(trk: Tracker, events: Sequence[tuple], grids: Sequence[int] = GRIDS,
             graphs: Sequence[int] = (0, 1), reps: int = 3, cache: Optional[str] = DEFAULT_CACHE,
             log=None) -> Dict:
    """Time every (tracklet_grid, use_graph) on `events` (list of cluster
    tensor tuples on one non-null stream for graph replay); apply and cache
    the fastest.  Returns {"best": {...}, "trials": [...]}."""
    n = sum(int(e[0].shape[0]) for e in events)
    key = _key(n, len(events))
    keep = trk.get_tuning()
    trials: List[Dict] = []
    for g in grids:
        for u in graphs:
            trk.set_tuning(ckpt_every=keep.ckpt_every, tracklet_grid=g, use_graph=u)
            t = time_config(trk, events, reps)
            trials.append(dict(tracklet_grid=g, use_graph=u, ms=t * 1e3))
            if log:
                log(f"autotune {key}: grid={g} graph={u} {t * 1e3:.3f} ms")
    best = min(trials, key=lambda d: d["ms"])
    trk.set_tuning(ckpt_every=keep.ckpt_every, tracklet_grid=best["tracklet_grid"],
                   use_graph=best["use_graph"])
    if cache:
        data = {}
        if os.path.exists(cache):
            try:
                data = json.load(open(cache))
            except (OSError, ValueError):
                data = {}
        data[key] = dict(best=best, trials=trials)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(key=key, best=best, trials=trials)


def load_tuning(trk: Tracker, n_clusters: int, n_events: int, cache: str = DEFAULT_CACHE) -> bool:
    """Apply a cached setting for this workload size if one exists."""
    if not os.path.exists(cache):
        return False
    try:
        data = json.load(open(cache))
    except (OSError, ValueError):
        return False
    ent = data.get(_key(n_clusters, n_events))
    if not ent:
        return False
    b = ent["best"]
    keep = trk.get_tuning()
    trk.set_tuning(ckpt_every=keep.ckpt_every, tracklet_grid=b["tracklet_grid"], use_graph=b["use_graph"])
    return True
