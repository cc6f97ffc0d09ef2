"""Continuous-batching request loop for jet solves.

Requests (a jet configuration, its inlet rows and a step count) arrive over
time.  A request is admitted as soon as it has arrived, a slot is free and
its two population buffers fit the HBM budget; its populations stay resident
on the device until it finishes.  All resident jets advance together, k
steps per group, in one persistent launch per step for each cohort of
jets (one storage form per cohort).  The loop queues each
group before it handles the previous one, so the device is not left idle
while the host works: the jets that reached their step count in the previous
group return their centreline and exit-column profiles of u_x and T and free
their slot and memory, and requests that arrived meanwhile are admitted and
join the next group queued.  FP16 requests of more than FP16_STEP_LIMIT steps
(by default every one) are stored with stochastic rounding (route), whose
temperature stays within 1e-3 of the oracle's up to 4 000 steps and within
3e-3 at 10 000.

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


# Runs longer than this go from FP16 storage to FP16 with stochastic rounding
# (route).  Rounding to nearest biases the temperature, whose profile error
# grows linearly in time: 1.3e-3 at 1 000 steps and 8.7e-3 at 4 000 on the
# jets of this workload, against 2.7e-4 and 7.0e-4 with stochastic rounding
# (tests/test_gpu_run_length.py).  With gfx950's rounding conversion a batch
# of FP16SR jets serves as many requests per second as one of FP16 jets, so
# by default every FP16 request is stored that way.
FP16_STEP_LIMIT = 0


def route(precision: str, steps: int, long_after: int = FP16_STEP_LIMIT,
          long_storage: str = "fp16sr") -> str:
    """The storage a request runs in: FP16 requests of more than `long_after`
    steps run in `long_storage` (long_after < 0: never)."""
    if precision == "fp16" and long_after >= 0 and steps > long_after:
        return long_storage
    return precision


def serve(requests, precision: str = "fp16", budget_bytes: int = 16 << 30,
          max_slots: int = 256, k_steps: int = 100, realtime: bool = True,
          tile_shape: int = -1, workgroups: int = 0, keep_profiles: bool = False,
          layout: str = "two", streams: int = 0, cohort_bytes: int = -1,
          long_after: int = FP16_STEP_LIMIT, long_storage: str = "fp16sr",
          pipeline: bool = True):
    """Run the request list [(arrival_s, params, inlet, steps), ...].
    layout="single" keeps each resident jet in one buffer updated in place,
    so a budget holds twice as many jets.

    Requests run in `precision`, except that with FP16 storage those of more
    than `long_after` steps run in `long_storage` (route): one batch holds
    both, each storage form in cohorts of its own.

    realtime=False admits every request at t = 0 (saturation: measures the
    capacity).  pipeline=False waits for each group before the host retires
    and admits (the device idles meanwhile).  streams (1 to 4) and
    cohort_bytes override the batch's defaults when given.  Returns a summary
    dict, plus per-request records.
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

        def finish(slots):
            nonlocal updates
            for slot in slots:
                q = live.pop(slot)
                prof = b.profiles(slot)  # waits for the group it finished in
                t_done = now()
                b.retire(slot)
                rec[q]["completed"] = t_done
                rec[q]["latency"] = t_done - rec[q]["arrival"]
                updates += rec[q]["nodes"] * rec[q]["steps"]
                if keep_profiles:
                    rec[q]["profiles"] = prof

        finished_prev = []  # slots of jets that finished in the last group queued
        host = collections.Counter()  # host seconds by phase
        while pending or live:
            t = now()
            while pending and (not realtime or requests[pending[0]][0] <= t):
                q = pending[0]
                arr, p, inlet, steps = requests[q]
                pr = route(precision, steps, long_after, long_storage)
                rc, slot = b.try_admit(p, inlet, steps, precision=pr)
                if rc == lbm.ENOMEM and not live:
                    raise lbm.LbmError(rc, "lbm_batch_admit",
                                       f"request {q} ({p['nx']} x {p['nr']}, {pr}) does not fit "
                                       "an empty batch: budget or slot count too small")
                if rc == lbm.ENOMEM:
                    break
                if rc != lbm.OK:
                    raise lbm.LbmError(rc, "lbm_batch_admit", lbm.strerror(rc))
                live[slot] = q
                pending.popleft()
                rec[q] = {"arrival": arr if realtime else 0.0, "admitted": now(),
                          "nodes": p["nx"] * p["nr"], "steps": steps, "storage": pr}
            n_act, used = b.active()
            peak_slots = max(peak_slots, n_act)
            peak_bytes = max(peak_bytes, used)
            running = [s for s, q in live.items() if b.poll(s) < rec[q]["steps"]]
            t1 = now()
            host["admit"] += t1 - t
            if running:
                # queue the next group first: the device runs it while the
                # host retires the jets of the previous group and admits
                b.run(k_steps)
                t2 = now()
                # the previous group (this one runs on), or this one when not
                # pipelined
                b.wait(1 if pipeline else 0)
                t3 = now()
                groups += 1
                finish(finished_prev)
                finished_prev = [s for s in running if b.poll(s) >= rec[live[s]]["steps"]]
                if not pipeline:
                    finish(finished_prev)
                    finished_prev = []
                host["run"] += t2 - t1
                host["wait"] += t3 - t2
                host["finish"] += now() - t3
            else:
                finish(finished_prev + [s for s in live if s not in finished_prev])
                finished_prev = []
                if pending and realtime:
                    time.sleep(max(0.0, min(requests[pending[0]][0] - now(), 0.01)))
        t_end = now()
        b.sync()
        dev_ms, dev_groups = b.device_time()
    lat = [r["latency"] for r in rec]
    first = min(r["arrival"] for r in rec)
    summary = {
        "requests": len(requests), "precision": precision, "realtime": realtime,
        "pipeline": pipeline,
        "storage_counts": dict(collections.Counter(r["storage"] for r in rec)),
        "k_steps": k_steps, "groups": groups,
        "p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4),
        # arrival to admission (queueing for memory or slots, and the group in flight)
        "admit_wait_p99_s": round(percentile([r["admitted"] - r["arrival"] for r in rec], 99), 4),
        "mean_s": round(float(np.mean(lat)), 4),
        "wall_s": round(t_end - first, 3),
        "requests_per_s": round(len(requests) / (t_end - first), 3),
        "glups": round(updates / (t_end - first) / 1e9, 3),
        "peak_slots": peak_slots, "peak_bytes": peak_bytes, "budget_bytes": budget_bytes,
        # host time per group, by phase: admitting, queueing the group, waiting
        # for the previous one, retiring the jets it finished
        "host_ms_per_group": {k: round(v / max(groups, 1) * 1e3, 3) for k, v in host.items()},
        # device time of the groups (HIP events around each group) over the
        # loop's wall time: the share of it in which the device ran a group
        "device_ms_per_group": round(dev_ms / max(dev_groups, 1), 3),
        "device_busy": round(dev_ms * 1e-3 / max(t_end, 1e-9), 4),
        "timed_groups": dev_groups,
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
    ap.add_argument("--tile-shape", type=int, default=-1,
                    help="tile shape index for every storage form (-1: the batch's default)")
    ap.add_argument("--cohort-mib", type=int, default=-1,
                    help="cohort limit in MiB (-1: the batch's default, 0: one cohort)")
    ap.add_argument("--sweep", default="",
                    help="comma-separated fractions of the measured capacity to run at "
                         "(e.g. 0.3,0.5,0.7,0.9); overrides --rate")
    ap.add_argument("--sync", action="store_true",
                    help="wait for each group before retiring and admitting")
    ap.add_argument("--long-after", type=int, default=FP16_STEP_LIMIT,
                    help="FP16 requests of more steps run in --long-storage (-1: never)")
    ap.add_argument("--long-storage", default="fp16sr", choices=["fp16sr", "fp32"])
    args = ap.parse_args()
    budget = int(args.budget_gb * (1 << 30))
    cohort = args.cohort_mib << 20 if args.cohort_mib >= 0 else -1
    rate = args.rate
    cap = None
    if rate <= 0 or args.sweep:
        cap, _ = serve(inputs.arrival_trace(args.requests, args.seed, rate=1.0), args.precision,
                       budget, args.slots, args.k, realtime=False, layout=args.layout,
                       streams=args.streams, cohort_bytes=cohort, long_after=args.long_after,
                       long_storage=args.long_storage, pipeline=not args.sync,
                       tile_shape=args.tile_shape)
        print(json.dumps({"saturated": cap}), flush=True)
    fractions = [float(x) for x in args.sweep.split(",") if x] if args.sweep else [None]
    for frac in fractions:
        if frac is not None:
            rate = frac * cap["requests_per_s"]
        elif rate <= 0:
            rate = 0.7 * cap["requests_per_s"]
        trace = inputs.arrival_trace(args.requests, args.seed, rate=rate)
        summary, _ = serve(trace, args.precision, budget, args.slots, args.k, realtime=True,
                           layout=args.layout, streams=args.streams, cohort_bytes=cohort,
                           long_after=args.long_after,
                           long_storage=args.long_storage, pipeline=not args.sync,
                           tile_shape=args.tile_shape)
        summary["rate"] = rate
        if frac is not None:
            summary["fraction_of_capacity"] = frac
        print(json.dumps({"poisson": summary}), flush=True)


if __name__ == "__main__":
    main()
