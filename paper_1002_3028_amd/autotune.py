"""Launch autotuner of the step kernels.

Single jets (best_shape): for a precision and a size class it times every
compiled tile shape (block shape, nodes per lane, cache policy, one or two
steps per launch) on a representative jet and keeps the fastest.  Size
classes follow the memory system: the two population buffers either fit the
256 MB Infinity Cache with room to spare, or do not.

Batches (tune_batch): for a set of jets advanced together it searches the
tile shape, the persistent grid, the cohort size and the number of streams.

Results are cached as JSON keyed by GPU architecture, precision and size
class in $LBM_AUTOTUNE_CACHE or ~/.cache/lbmx/autotune.json.
"""
from __future__ import annotations

import json
import os
import time

from . import lbm

MALL_BYTES = 200 << 20  # buffers below this stay resident in the Infinity Cache


def cache_path() -> str:
    return os.environ.get("LBM_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "lbmx", "autotune.json")


def size_class(working_set_bytes: int) -> str:
    if working_set_bytes < (16 << 20):
        return "small"
    return "cache" if working_set_bytes < MALL_BYTES else "hbm"


def _arch() -> str:
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(d: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def time_shapes(params: dict, inlet, precision: str, steps: int = 200, warmup: int = 30,
                shapes=None, graph_steps: int = 50, rounds: int = 2) -> dict:
    """Seconds per step of each tile shape on one jet (shape index -> s): the
    fastest of `rounds` passes over the shapes, every other pass in reverse
    order, so that no shape is timed only while the device warms up."""
    import torch
    out = {}
    order = list(range(len(lbm.tile_shapes())) if shapes is None else shapes)
    with lbm.Solver(params, precision, graph_steps=graph_steps) as s:
        if inlet is not None:
            s.set_inlet(*inlet)
        for q in [q for r in range(rounds) for q in (order if r % 2 == 0 else order[::-1])]:
            try:
                s.set_tile_shape(q)
            except lbm.LbmError as e:  # a shape this handle cannot take
                if e.code != lbm.EINVAL:
                    raise
                continue
            s.step(warmup)
            s.sync()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.torch_stream)
            s.step(steps)
            e1.record(s.torch_stream)
            s.sync()
            t = e0.elapsed_time(e1) * 1e-3 / steps
            out[q] = min(out.get(q, t), t)
    return out


def best_shape(params: dict, inlet, precision: str, retune: bool = False,
               steps: int | None = None) -> int:
    """Fastest tile shape for this jet's size class (tuned once, cached);
    steps = 1 or 2 restricts the choice to shapes taking that many steps per
    launch."""
    ws = lbm.bytes_required(params, precision)
    key = f"{_arch()}/{precision}/{size_class(ws)}"
    periodic = "periodic" in tuple(params.get("bc", ()))[:2]
    if periodic:
        key += "/periodic"
    if steps is not None:
        key += f"/steps{steps}"
    db = _load()
    infos = lbm.tile_shape_infos()
    hit = db.get(key)
    if hit is not None and not retune and hit.get("info") in infos:
        return infos.index(hit["info"])
    cand = [q for q, inf in enumerate(infos) if steps is None or inf["steps"] == steps]
    t = time_shapes(params, inlet, precision, shapes=cand)
    q = min(t, key=t.get)
    db[key] = {"info": infos[q], "s_per_step": t[q], "tuned_on": [params["nx"], params["nr"]],
               "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    _save(db)
    return q


# search space of the batch tuner (coordinate descent, stage by stage)
BATCH_WORKGROUPS = (0, 1024, 2048, 4096, 8192)  # 0: the device's resident count
BATCH_COHORT_MIB = (64, 96, 112, 128, 160, 200, 0)  # 0: all jets in one cohort
BATCH_STREAMS = (1, 2, 3)


def batch_key(jets, precision: str) -> str:
    """Cache key of a set of jets: precision, jet count and total population
    bytes (to the nearest power of two) -- the two things the best cohort
    split and grid depend on."""
    import math
    total = sum(lbm.bytes_required(p, precision) for p, _ in jets)
    return (f"{_arch()}/{precision}/batch/{len(jets)}jets/"
            f"{2 ** round(math.log2(max(total, 1 << 20)) - 20)}MiB")


def apply_batch(b, cfg: dict) -> None:
    """Put a tuned configuration (from tune_batch) on an lbm.Batch."""
    b.set_launch(cfg["shape"], cfg["workgroups"])
    b.set_cohort_bytes(cfg["cohort_mib"] << 20)
    b.set_streams(cfg["streams"])


def _time_batch(b, k_steps, rounds):
    """Seconds per step of the batch's current configuration: one warm group
    (captures its graphs), then the fastest of `rounds` timed groups."""
    b.run(k_steps)
    b.sync()
    best = None
    for _ in range(rounds):
        t0 = time.perf_counter()
        b.run(k_steps)
        b.sync()
        dt = (time.perf_counter() - t0) / k_steps
        best = dt if best is None else min(best, dt)
    return best


def tune_batch(jets, precision: str, retune: bool = False, k_steps: int = 50,
               rounds: int = 3, shapes=None) -> dict:
    """Fastest launch configuration for a set of jets advanced together in
    one batch: tile shape, persistent workgroups, cohort size and number of
    streams.  jets: list of (params, inlet).

    Coordinate descent over the compiled tile shapes (with the batch's
    default grid, cohorts and streams), then the grid, then cohort size and
    stream count together, each stage keeping the best of the previous.  The
    result is cached under batch_key (tuned once per GPU architecture,
    precision and size class of the set) and returned as a dict for
    apply_batch.  Every configuration gives the same bits; only the time
    differs."""
    key = batch_key(jets, precision)
    db = _load()
    infos = lbm.tile_shape_infos()
    hit = db.get(key)
    if hit is not None and not retune and hit.get("info") in infos:
        cfg = dict(hit["config"])
        cfg["shape"] = infos.index(hit["info"])
        return cfg
    budget = sum(lbm.bytes_required(p, precision) for p, _ in jets) + (64 << 20)
    times = {}
    with lbm.Batch(budget, len(jets), precision) as b:
        for p, inlet in jets:
            b.admit(p, inlet, 1 << 40)
        cfg = {"shape": -1, "workgroups": 0, "cohort_mib": 128, "streams": 2}

        def trial(**change):
            c = dict(cfg, **change)
            apply_batch(b, c)
            t = _time_batch(b, k_steps, rounds)
            times[json.dumps(c, sort_keys=True)] = t
            return t, c

        cand = range(len(infos)) if shapes is None else shapes
        best = min((trial(shape=q) for q in cand), key=lambda tc: tc[0])
        cfg = best[1]
        best = min([best] + [trial(workgroups=w) for w in BATCH_WORKGROUPS
                             if w != cfg["workgroups"]], key=lambda tc: tc[0])
        cfg = best[1]
        best = min([best] + [trial(cohort_mib=m, streams=n) for m in BATCH_COHORT_MIB
                             for n in BATCH_STREAMS
                             if (m, n) != (cfg["cohort_mib"], cfg["streams"])],
                   key=lambda tc: tc[0])
        cfg = best[1]
    out = dict(cfg, s_per_step=best[0], trials=len(times))
    db[key] = {"info": infos[cfg["shape"]], "config": {k: v for k, v in out.items()
                                                       if k != "shape"},
               "tuned_on": len(jets), "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    _save(db)
    return out
