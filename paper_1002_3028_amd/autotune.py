"""Launch-shape autotuner for the step kernel.

For a precision and a size class it times every compiled tile shape (block
shape, nodes per lane, cache policy, one or two steps per launch) on a
representative jet and keeps the fastest.  Results are cached as JSON keyed by (GPU architecture, precision,
size class) in $LBM_AUTOTUNE_CACHE or ~/.cache/lbmx/autotune.json.

Size classes follow the memory system: the two population buffers either
fit the 256 MB Infinity Cache with room to spare, or do not.
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
                shapes=None, graph_steps: int = 50) -> dict:
    """Seconds per step of each tile shape on one jet (shape index -> s)."""
    import torch
    out = {}
    with lbm.Solver(params, precision, graph_steps=graph_steps) as s:
        if inlet is not None:
            s.set_inlet(*inlet)
        for q in (range(len(lbm.tile_shapes())) if shapes is None else shapes):
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
            out[q] = e0.elapsed_time(e1) * 1e-3 / steps
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


def tune_batch(jets, precision: str, budget_bytes: int, k_steps: int = 20, rounds: int = 2,
               workgroups=(1024, 2048, 4096, 8192)):
    """Fastest (tile shape, persistent workgroups) for a set of jets advanced
    together.  jets: list of (params, inlet).  Returns (shape, workgroups, s)."""
    import torch
    best = None
    with lbm.Batch(budget_bytes, len(jets), precision) as b:
        for p, inlet in jets:
            b.admit(p, inlet, 1 << 40)
        for q in range(len(lbm.tile_shapes())):
            for wg in workgroups:
                b.set_launch(q, wg)
                b.run(k_steps)
                b.sync()
                t0 = time.perf_counter()
                for _ in range(rounds):
                    b.run(k_steps)
                b.sync()
                dt = (time.perf_counter() - t0) / (rounds * k_steps)
                if best is None or dt < best[2]:
                    best = (q, wg, dt)
    return best
