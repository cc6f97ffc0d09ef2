"""Measurement probe for hardware counters.

Runs, on the current device: a plain copy of a known size (the calibration
of the HBM traffic counters), then the step kernel of one workload with one
launch per step (no graphs), so that a counter collection sees one dispatch
per step.  The batch64 workload runs the 64 uneven jets of the batch
benchmark in one batch (default cohorts, one stream) for --steps steps and
prints the number of cohorts, so that bytes per launch can be set against
the cohort's average node count.

  python -m paper_1002_3028_amd.probe --workload single --precision fp32
"""
from __future__ import annotations

import argparse

from . import inputs, lbm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["single", "large", "batch64"], default="single")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=256)
    ap.add_argument("--tile-shape", type=int, default=-1)
    ap.add_argument("--layout", choices=["two", "single"], default="two")
    args = ap.parse_args()
    import torch

    n = args.copy_mib << 20
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.Stream()
    for _ in range(3):
        lbm.probe_copy(b.data_ptr(), a.data_ptr(), n, st.cuda_stream)
    st.synchronize()
    del a, b
    print(f"copy calibration: 3 x {args.copy_mib} MiB", flush=True)
    if args.workload == "batch64":
        batch64(args)
        return
    if args.workload == "single":
        p, inlet, _ = inputs.workload_single(n_t=max(1, args.steps))
    else:
        p, inlet, _ = inputs.workload_large(n_t=max(1, args.steps))
    kw = {} if args.tile_shape < 0 else {"tile_shape": args.tile_shape}
    with lbm.Solver(p, args.precision, layout=args.layout, **kw) as s:
        s.set_inlet(*inlet)
        s.step(args.steps)
        s.sync()
    print(f"step kernel: {p['nx']}x{p['nr']} {args.precision}, {args.steps} launches", flush=True)


def batch64(args):
    """The 64-jet batch of the benchmark, one stream, default cohorts."""
    jets = inputs.batch_jets(64, seed=2, steps=args.steps)
    nodes = sum(p["nx"] * p["nr"] for p, _, _ in jets)
    budget = sum(lbm.bytes_required(p, args.precision) for p, _, _ in jets) + (64 << 20)
    with lbm.Batch(budget, 64, args.precision) as b:
        b.set_streams(1)
        if args.tile_shape >= 0:
            b.set_launch(args.tile_shape, 0)
        for p, inlet, _ in jets:
            b.admit(p, inlet, args.steps + 100)
        # the runtime's grouping: slot order, a new cohort whenever the next
        # jet would take the current one past the limit
        limit, cohorts, cur = 128 << 20, 1, 0
        for p, _, _ in jets:
            jb = b.jet_bytes(p)
            if cur and cur + jb > limit:
                cohorts, cur = cohorts + 1, 0
            cur += jb
        b.run(args.steps)
        b.sync()
    print(f"batch: 64 jets, {nodes} nodes, {cohorts} cohorts, {args.steps} steps "
          f"({args.precision}), {nodes // cohorts} nodes per launch on average", flush=True)


if __name__ == "__main__":
    main()
