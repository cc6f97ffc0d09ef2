"""Writes the FP64 oracle's end-of-run profiles of four jets of the serving
workload at several run lengths (tests/golden/serving_profiles.txt), against
which the GPU test measures each storage form's profile error as a function
of the number of steps.

Calls only the oracle and the seeded input generator.  The jets are the
first request of the serving trace (seed 3) whose axial size falls in each
of [128, 256), [256, 512), [512, 1024) and [1024, 2048]; each runs from the
ambient rest state with its own parameters (parabolic inlet of eq. 7, no
noise) for 10 000 steps.  At steps 1000, 2000, 4000 and 10 000 the file holds
what a serving request returns: the centreline (j = 0) u_x and T and the
exit-column (i = nx - 1) u_x and T.

Usage: python tests/golden/make_serving_profiles.py [--threads N]
(about 8 minutes on 8 cores).
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CHECKPOINTS = (1000, 2000, 4000, 10000)
BANDS = ((128, 256), (256, 512), (512, 1024), (1024, 2049))


def jets():
    """[(trace index, params, inlet)] for the four size bands."""
    from paper_1002_3028_amd import inputs
    trace = inputs.arrival_trace(2000, 3, rate=1.0)
    out = []
    for lo, hi in BANDS:
        q = next(q for q, (_, p, _, _) in enumerate(trace) if lo <= p["nx"] < hi)
        out.append((q, trace[q][1], trace[q][2]))
    return out


def write(path, records):
    with open(path + ".tmp", "w") as fh:
        fh.write("# FP64 oracle, serving-trace jets (seed 3): end-of-run profiles\n")
        fh.write("# written by tests/golden/make_serving_profiles.py (oracle only)\n")
        for (q, steps), prof in records.items():
            for k, v in prof.items():
                fh.write(f"{q} {steps} {k} {v.size}\n")
                for x in v:
                    fh.write(f"{x:.17g}\n")
    os.replace(path + ".tmp", path)


def read(path):
    """{(trace index, steps): {name: array}}."""
    out = {}
    with open(path) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    i = 0
    while i < len(lines):
        q, steps, key, n = lines[i].split()
        n = int(n)
        out.setdefault((int(q), int(steps)), {})[key] = np.array(
            [float(x) for x in lines[i + 1:i + 1 + n]])
        i += 1 + n
    return out


def main():
    import oracle

    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    records = {}
    for q, p, inlet in jets():
        t0 = time.time()
        with oracle.RefSolver(p, threads=args.threads) as r:
            r.set_inlet(*inlet)
            done = 0
            for c in CHECKPOINTS:
                r.step(c - done)
                done = c
                records[(q, c)] = r.profiles()
                print(f"request {q} ({p['nx']}x{p['nr']}): step {c}, {time.time() - t0:.0f} s",
                      flush=True)
    write(os.path.join(HERE, "serving_profiles.txt"), records)


if __name__ == "__main__":
    main()
