"""Continuous-batching request loop for jet solves.

Requests (a jet configuration, its inlet rows and a step count) arrive over
time.  A request is admitted as soon as it has arrived, a slot is free and
its two population buffers fit the HBM budget; its populations stay resident
on the device until it finishes.  All resident jets advance together, k
steps per group, in one persistent launch per step.  After each group the
jets that reached their step count return their centreline and exit-column
profiles of u_x and T and free their slot and memory, so requests that
arrived meanwhile join the next group.

Latency is completion minus arrival (wall clock); completion is taken when
the device has finished the group in which the jet reached its step count.

Run as a module for the 2000-request trace:
  python -m paper_1002_3028_amd.serve --requests 2000 --rate 40 --precision fp16
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import time

import numpy as np

from . import inputs, lbm


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else math.nan


def serve(requests, precision: str = "fp16", budget_bytes: int = 16 << 30,
          max_slots: int = 256, k_steps: int = 100, realtime: bool = True,
          tile_shape: int = -1, workgroups: int = 0, keep_profiles: bool = False,
          layout: str = "two", streams: int = 0, cohort_bytes: int = -1):
    """Run the request list [(arrival_s, params, inlet, steps), ...].
    layout="single" keeps each resident jet in one buffer updated in place,
    so a budget holds twice as many jets.

    realtime=False admits every request at t = 0 (saturation: measures the
    capacity).  streams (1 to 4) and cohort_bytes override the batch's
    defaults when given.  Returns a summary dict, plus per-request records.
    """
    order = sorted(range(len(requests)), key=lambda q: requests[q][0])
    pending = collections.deque(order)
    live = {}  # slot -> request index
    rec = [None] * len(requests)
    updates = 0
    groups = 0
    peak_slots = 0
    peak_bytes = 0
    with lbm.Batch(budget_bytes, max_slots, precision, layout=layout) as b:
        b.set_launch(tile_shape, workgroups)
        if streams:
            b.set_streams(streams)
        if cohort_bytes >= 0:
            b.set_cohort_bytes(cohort_bytes)
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        while pending or live:
            t = now()
            while pending and (not realtime or requests[pending[0]][0] <= t):
                q = pending[0]
                arr, p, inlet, steps = requests[q]
                rc, slot = b.try_admit(p, inlet, steps)
                if rc == lbm.ENOMEM:
                    break
                if rc != lbm.OK:
                    raise lbm.LbmError(rc, "lbm_batch_admit", lbm.strerror(rc))
                live[slot] = q
                pending.popleft()
                rec[q] = {"arrival": arr if realtime else 0.0, "admitted": now(),
                          "nodes": p["nx"] * p["nr"], "steps": steps}
            n_act, used = b.active()
            peak_slots = max(peak_slots, n_act)
            peak_bytes = max(peak_bytes, used)
            if not live:
                if pending and realtime:
                    time.sleep(max(0.0, min(requests[pending[0]][0] - now(), 0.01)))
                continue
            b.run(k_steps)
            groups += 1
            done = [s for s, q in live.items() if b.poll(s) >= rec[q]["steps"]]
            b.sync()
            t_done = now()
            for s in done:
                q = live.pop(s)
                prof = b.profiles(s)
                b.retire(s)
                rec[q]["completed"] = t_done
                rec[q]["latency"] = t_done - rec[q]["arrival"]
                updates += rec[q]["nodes"] * rec[q]["steps"]
                if keep_profiles:
                    rec[q]["profiles"] = prof
        t_end = now()
    lat = [r["latency"] for r in rec]
    first = min(r["arrival"] for r in rec)
    summary = {
        "requests": len(requests), "precision": precision, "realtime": realtime,
        "k_steps": k_steps, "groups": groups,
        "p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4),
        "mean_s": round(float(np.mean(lat)), 4),
        "wall_s": round(t_end - first, 3),
        "requests_per_s": round(len(requests) / (t_end - first), 3),
        "glups": round(updates / (t_end - first) / 1e9, 3),
        "peak_slots": peak_slots, "peak_bytes": peak_bytes, "budget_bytes": budget_bytes,
    }
    return summary, rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=0.0,
                    help="Poisson rate (requests/s); 0: 0.7 x the measured capacity")
    ap.add_argument("--precision", default="fp16")
    ap.add_argument("--budget-gb", type=float, default=16.0)
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--layout", choices=["two", "single"], default="two")
    ap.add_argument("--streams", type=int, default=0, help="1 to 4 (0: the batch's default)")
    ap.add_argument("--cohort-mib", type=int, default=-1,
                    help="cohort limit in MiB (-1: the batch's default, 0: one cohort)")
    ap.add_argument("--sweep", default="",
                    help="comma-separated fractions of the measured capacity to run at "
                         "(e.g. 0.3,0.5,0.7,0.9); overrides --rate")
    args = ap.parse_args()
    budget = int(args.budget_gb * (1 << 30))
    cohort = args.cohort_mib << 20 if args.cohort_mib >= 0 else -1
    rate = args.rate
    cap = None
    if rate <= 0 or args.sweep:
        cap, _ = serve(inputs.arrival_trace(args.requests, args.seed, rate=1.0), args.precision,
                       budget, args.slots, args.k, realtime=False, layout=args.layout,
                       streams=args.streams, cohort_bytes=cohort)
        print(json.dumps({"saturated": cap}), flush=True)
    fractions = [float(x) for x in args.sweep.split(",") if x] if args.sweep else [None]
    for frac in fractions:
        if frac is not None:
            rate = frac * cap["requests_per_s"]
        elif rate <= 0:
            rate = 0.7 * cap["requests_per_s"]
        trace = inputs.arrival_trace(args.requests, args.seed, rate=rate)
        summary, _ = serve(trace, args.precision, budget, args.slots, args.k, realtime=True,
                           layout=args.layout, streams=args.streams, cohort_bytes=cohort)
        summary["rate"] = rate
        if frac is not None:
            summary["fraction_of_capacity"] = frac
        print(json.dumps({"poisson": summary}), flush=True)


if __name__ == "__main__":
    main()
