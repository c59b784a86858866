"""Launch-shape autotuner for the batch simulation.

Times candidate tuning keys (persistent work-groups, LDS-resident queue
blocks per DAG) on the caller's own workload and caches the fastest per
(device architecture, CU count, workload signature).  Every key yields the
same schedule; only the time differs.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np


def _cache_path():
    return os.environ.get("INSP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "inspirit",
                                                           "tune.json"))


def signature(dag, workers, prm) -> str:
    h = hashlib.sha1()
    h.update(np.asarray(dag.n, np.int64).tobytes())
    h.update(np.asarray(dag.m, np.int64).tobytes())
    h.update(np.asarray(workers, np.int32).tobytes())
    h.update(np.asarray([prm.policy, prm.attr_mode, prm.data_bw], np.int64).tobytes())
    return h.hexdigest()[:16]


def candidates(n_dags, cus):
    # three work-groups per CU with more LDS-resident queue blocks (keys of
    # further blocks beside full entries), or four with fewer
    grids = sorted({min(n_dags, cus * k) for k in (3, 4)})
    shapes = ("lds_blocks=256,lds_slots=16", "lds_blocks=256,lds_slots=24", "lds_blocks=128,lds_slots=32",
              "lds_blocks=128,lds_slots=24,lds_keys=40", "lds_blocks=128,lds_slots=16,lds_keys=48")
    return [f"grid={g},{sh}" for g in grids for sh in shapes]


def tune(dag, workers, dur, est, prm, out, reps=2, use_cache=True, verbose=False) -> str:
    """Candidates differ by a few percent, about the run-to-run spread, so
    each is scored by its fastest of `reps` single runs, and the best three
    are timed again in interleaved rounds before one is kept."""
    import torch
    from . import inspirit
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "gfx?")
    key = f"{arch}:{props.multi_processor_count}:{signature(dag, workers, prm)}"
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return cache[key]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def fastest(cand, runs):
        t = float("inf")
        for _ in range(runs):
            e0.record()
            inspirit.schedule_batch(dag, workers, dur, est, prm, tune_key=cand, out=out)
            e1.record()
            torch.cuda.synchronize()
            t = min(t, e0.elapsed_time(e1))
        return t

    cands = candidates(dag.n_dags, props.multi_processor_count)
    ms = {}
    for cand in cands:
        inspirit.schedule_batch(dag, workers, dur, est, prm, tune_key=cand, out=out)  # first use allocates
        torch.cuda.synchronize()
        ms[cand] = fastest(cand, reps)
    top = sorted(cands, key=ms.get)[:3]
    for _ in range(3):
        for cand in top:
            ms[cand] = min(ms[cand], fastest(cand, 1))
    best = min(top, key=ms.get)
    if verbose:
        for cand in cands:
            print(f"[tune] {cand}: {ms[cand]:.2f} ms", flush=True)
    cache[key] = best
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return best
