"""Measurement probe for hardware counters.

Runs, on the current device: a plain copy of a known size (the calibration
of the HBM traffic counters), then the step kernel of one workload with one
launch per step (no graphs), so that a counter collection sees one dispatch
per step.

  python -m paper_1002_3028_amd.probe --workload single --precision fp32
"""
from __future__ import annotations

import argparse

from . import inputs, lbm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["single", "large"], default="single")
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


if __name__ == "__main__":
    main()
