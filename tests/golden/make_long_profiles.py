"""Writes the FP64 oracle's time-averaged jet profiles that the long-run GPU
parity test compares against (tests/golden/long_profiles_<nx>x<nr>.txt).

Calls only the oracle and the seeded input generator (which holds none of the
method's arithmetic).  What is stored, for each jet:

* an N = 20 000-step run of the oracle from the ambient rest state, with the
  jet's inlet rows (one row per step, eq. 7 profiles with 1 % noise);
* time averages over steps [N/2, N], sampled every 50 steps (201 samples), of
  the centreline (j = 0) u_x(x) and T(x) and of the radial u_x(r), T(r) at
  i = nx/2 and i = nx - 1 -- the profiles the paper compares in its
  validation figures (section 4.1), here in lattice units.

Jets: the 2048 x 512 benchmark jet (radius 32, U_max 0.08, C_s 0.17, property
tables of seed 1) and the 1024 x 256 twin of the 4096 x 1024 jet (radius 16).

Usage: python tests/golden/make_long_profiles.py [--threads N] [--only NXxNR]
(about 20 minutes for both on 8 cores).
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_STEPS, EVERY = 20000, 50


def cuts(m):
    """Centreline and the two radial cuts of the moment fields."""
    nx = m["ux"].shape[1]
    return {"ux_axis": m["ux"][0], "T_axis": m["T"][0],
            "ux_mid": m["ux"][:, nx // 2], "T_mid": m["T"][:, nx // 2],
            "ux_exit": m["ux"][:, -1], "T_exit": m["T"][:, -1]}


def averaged(solver, name, steps=N_STEPS, every=EVERY):
    t0 = time.time()
    chunk = 1000
    for q in range(steps // 2 // chunk):
        solver.step(chunk)
        print(f"{name}: step {(q + 1) * chunk}, {time.time() - t0:.0f} s", flush=True)
    rest = steps // 2 - (steps // 2 // chunk) * chunk
    if rest:
        solver.step(rest)
    acc, n = None, 0
    for q in range(steps // 2 // every + 1):
        c = cuts(solver.moments())
        acc = c if acc is None else {k: acc[k] + c[k] for k in acc}
        n += 1
        if q < steps // 2 // every:
            solver.step(every)
    print(f"{name}: done, {time.time() - t0:.0f} s", flush=True)
    return {k: v / n for k, v in acc.items()}


def write(path, name, p, prof, steps, every):
    with open(path + ".tmp", "w") as fh:
        fh.write(f"# FP64 oracle, {name} jet: time averages over steps [{steps // 2}, {steps}] "
                 f"sampled every {every} steps ({steps // 2 // every + 1} samples)\n")
        fh.write(f"# nx {p['nx']} nr {p['nr']} steps {steps} every {every}\n")
        fh.write("# written by tests/golden/make_long_profiles.py (oracle only)\n")
        for k, v in prof.items():
            fh.write(f"{k} {v.size}\n")
            for x in v:
                fh.write(f"{x:.17g}\n")
    os.replace(path + ".tmp", path)


def read(path):
    """{name: array} from a file written by write()."""
    out = {}
    with open(path) as fh:
        lines = [ln for ln in fh if not ln.startswith("#")]
    q = 0
    while q < len(lines):
        key, n = lines[q].split()
        n = int(n)
        out[key] = np.array([float(x) for x in lines[q + 1:q + 1 + n]])
        q += 1 + n
    return out


def jets():
    from paper_1002_3028_amd import inputs
    p1, in1, _ = inputs.workload_single(n_t=N_STEPS)
    p2, in2, _ = inputs.workload_large(nx=1024, nr=256, n_t=N_STEPS)
    return {"2048x512": (p1, in1), "1024x256": (p2, in2)}


def main():
    import oracle

    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    for name, (p, inlet) in jets().items():
        if args.only and name != args.only:
            continue
        with oracle.RefSolver(p, threads=args.threads) as r:
            r.set_inlet(*inlet)
            prof = averaged(r, name)
        write(os.path.join(HERE, f"long_profiles_{name}.txt"), name, p, prof, N_STEPS, EVERY)


if __name__ == "__main__":
    main()
