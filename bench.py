"""Benchmark of the axisymmetric D2Q9 + D2Q4 LBGK-LES step on one MI355X.

A step is one time step of the whole hot path (edge pulls, moments,
properties, Smagorinsky relaxation time, sources, collision, store) over the
2048 x 512 jet; the FP64 conservation check runs once per 1000 steps inside
the timed region.  Throughput is GLUPS (lattice node updates per second /
1e9).  The roofline is HBM bandwidth at the algorithmic 104 B per node update
for FP32 storage (13 populations read and written) and 52 B for 16-bit
storage: `achieved` = those bytes times the node updates of one launch,
divided by the launch duration measured with HIP events.  A launch of the
LDS-blocked kernel performs two node updates per node while it reads and
writes each population once; the HBM bytes it actually moves (rocprofv3
counters) are reported beside it as `traffic`, and their rate as
`dram_GBps`.

Prints one JSON line.  Also reports FP16- and BF16-deviation storage on the
same jet, the 4096 x 1024 jet (a working set above the 256 MB Infinity
Cache), and the FP64 oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"fp32": 104, "fp16": 52, "bf16": 52, "fp16sr": 52}
# Vector ALU issue: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz (a wave64 FP32
# instruction every 4 cycles per SIMD; packed FP32 not used), lane-ops/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions in the collision of one FP32 node update as compiled for
# gfx950 (eqs. 2-6 and 1 from the pulled values to the relaxed ones; the
# counters' executed figure per kernel is read from profiles/valu_*.txt).
VALU_COLLISION = 185


def _ensure_built():
    from paper_1002_3028_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def kernel_of(info):
    return "pair_kernel" if info["steps"] == 2 else "step_kernel"


def read_summary(name, key):
    """A value from a committed counter summary under profiles/, or None when
    absent or taken on another version of the kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    from paper_1002_3028_amd.profsum import kernel_source_sha256
    if vals.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def read_traffic(name):
    """Per-launch HBM bytes (read + write) from a committed counter summary."""
    return read_summary(name, "hbm_bytes_per_launch")


def alu_roofline(kernel, nodes, ms_step):
    """The launch against vector-ALU issue: VALU instructions executed per
    node update (SQ_INSTS_VALU over SQ_WAVES from the committed counter
    summary of this kernel; null when stale) x node updates per second, and
    the collision's own instruction count beside it."""
    kind = kernel.split("_")[0]
    executed = read_summary(f"valu_{kind}_fp32_2048x512.txt", "valu_per_node_update")
    out = {"unit": "T lane-op/s", "peak": round(VALU_PEAK_TOPS, 2),
           "valu_collision_per_node_update": VALU_COLLISION,
           "valu_executed_per_node_update": executed, "achieved": None, "frac": None}
    if executed:
        achieved = executed * nodes / (ms_step * 1e-3) / 1e12
        out.update(achieved=round(achieved, 2), frac=round(achieved / VALU_PEAK_TOPS, 4))
    return out


def time_jet(params, inlet, precision, steps, warmup, graph_steps=50, check_every=1000,
             tile_shape=None, layout="two"):
    """Returns (seconds for `steps` steps, ms per step from HIP events on the
    solver's stream, 3-D mass from the FP64 check)."""
    import torch
    from paper_1002_3028_amd import lbm

    with lbm.Solver(params, precision, graph_steps=graph_steps, tile_shape=tile_shape,
                    layout=layout) as s:
        s.set_inlet(*inlet)
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(s.torch_stream)
        done = 0
        while done < steps:
            n = min(check_every, steps - done)
            s.step(n)
            done += n
        ev1.record(s.torch_stream)
        mass, energy = s.conservation()  # FP64 reduction + stability check (syncs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ev_ms = ev0.elapsed_time(ev1)
    return t1 - t0, ev_ms / steps, mass


def bench_batch(n_jets=64, steps=500, precision="fp32"):
    """64 jets of uneven sizes (seed 2) advanced together in one persistent
    launch per step, against the same jets run one after another through the
    single-jet path (same kernel).  Aggregate GLUPS of both."""
    import torch
    from paper_1002_3028_amd import inputs, lbm

    jets = inputs.batch_jets(n_jets, seed=2, steps=steps)
    nodes = sum(p["nx"] * p["nr"] for p, _, _ in jets)
    budget = sum(lbm.bytes_required(p, precision) for p, _, _ in jets) + (64 << 20)
    with lbm.Batch(budget, n_jets, precision) as b:
        for p, inlet, _ in jets:
            b.admit(p, inlet, steps + 100)
        b.run(50)
        b.sync()
        t0 = time.perf_counter()
        for _ in range(steps // 50):
            b.run(50)
        b.sync()
        t_batch = time.perf_counter() - t0
    solvers = []
    for p, inlet, _ in jets:
        s = lbm.Solver(p, precision, graph_steps=50)
        s.set_inlet(*inlet)
        s.step(50)
        solvers.append(s)
    torch.cuda.synchronize()
    for s in solvers:
        s.sync()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(steps)
        s.sync()
    t_loop = time.perf_counter() - t0
    for s in solvers:
        s.close()
    upd = nodes * (steps // 50) * 50
    return {"jets": n_jets, "nodes": nodes, "steps": (steps // 50) * 50, "precision": precision,
            "batched_glups": round(upd / t_batch / 1e9, 3),
            "looped_single_glups": round(nodes * steps / t_loop / 1e9, 3)}


def bench_serving(n_requests=200, precision="fp16"):
    """Poisson trace (seed 3): capacity with every request admitted at once,
    then p50/p99 latency at 0.7 x that rate."""
    from paper_1002_3028_amd import inputs, serve

    cap, _ = serve.serve(inputs.arrival_trace(n_requests, 3, rate=1.0), precision,
                         16 << 30, 256, 100, realtime=False)
    rate = 0.7 * cap["requests_per_s"]
    run, _ = serve.serve(inputs.arrival_trace(n_requests, 3, rate=rate), precision,
                         16 << 30, 256, 100, realtime=True)
    return {"requests": n_requests, "precision": precision,
            "capacity_req_per_s": cap["requests_per_s"], "capacity_glups": cap["glups"],
            "rate_req_per_s": round(rate, 3), "p50_s": run["p50_s"], "p99_s": run["p99_s"],
            "glups_at_rate": run["glups"]}


def copy_ceiling(nbytes, reps=50):
    """A plain 16-byte-per-lane copy of nbytes into another nbytes (read +
    write = 2 nbytes moved), timed with HIP events: the streaming rate a
    kernel that reads one buffer and writes another can hope for."""
    import torch
    from paper_1002_3028_amd import lbm

    nbytes = nbytes // 256 * 256
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        lbm.probe_copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        lbm.probe_copy(b.data_ptr(), a.data_ptr(), nbytes, st.cuda_stream)
    e1.record(st)
    st.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_buffer": nbytes, "us": round(ms * 1e3, 2),
            "GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def cpu_baseline(params, inlet, budget_s=12.0):
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    nodes = params["nx"] * params["nr"]
    with oracle.RefSolver(params, threads=threads) as ref:
        ref.set_inlet(*inlet)
        t = time.perf_counter()
        ref.step(2)
        per = (time.perf_counter() - t) / 2
        n = int(max(4, min(4000, budget_s / per)))
        t = time.perf_counter()
        ref.step(n)
        dt = time.perf_counter() - t
    return {"value": round(nodes * n / dt / 1e9, 6), "unit": "GLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{params['nx']}x{params['nr']} jet, steps 2..{n + 2} from rest "
                      f"(FP64, OpenMP over radial rows), {dt:.1f} s"}


def oracle_timing():
    """The FP64 oracle on one thread and on every host core (OpenMP over radial
    rows; bit-identical results for any thread count): the 128 x 32 jet for
    its 500 steps, the first 200 steps of the 2048 x 512 jet and 100 steps of
    the 1024 x 256 twin of the 4096 x 1024 jet, warm (after two steps), median
    of three for runs under a second."""
    import platform
    import oracle
    from paper_1002_3028_amd import inputs

    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")),
                         "")
    except OSError:
        pass
    cores = max(1, min(16, os.cpu_count() or 1))
    cases = [("128x32 jet, 500 steps", inputs.workload_small()[:2], 500),
             ("2048x512 jet, first 200 steps", inputs.workload_single(n_t=200)[:2], 200),
             ("1024x256 twin, 100 steps", inputs.workload_large(1024, 256, n_t=100)[:2], 100)]
    rows = []
    for name, (p, inlet), steps in cases:
        nodes = p["nx"] * p["nr"]
        for threads in (1, cores):
            times = []
            for _ in range(3):
                with oracle.RefSolver(p, threads=threads) as ref:
                    ref.set_inlet(*inlet)
                    ref.step(2)
                    t = time.perf_counter()
                    ref.step(steps)
                    times.append(time.perf_counter() - t)
                if times[-1] > 1.0:
                    break
            dt = sorted(times)[len(times) // 2]
            rows.append({"case": name, "threads": threads, "seconds": round(dt, 3),
                         "mlups": round(nodes * steps / dt / 1e6, 2)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"oracle_timing": rows,
            "host": {"cpu": model, "nproc": os.cpu_count(), "machine": platform.machine(),
                     "compiler": "gcc -O2 -std=c11 -ffp-contract=off -fopenmp"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle (1 thread and all cores) and exit")
    args = ap.parse_args()
    if args.oracle_timing:
        print(json.dumps(oracle_timing()))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1 (jets are "
                          "independent, so several GPUs would each run their own share)"}))
        sys.exit(2)

    import torch
    from paper_1002_3028_amd import autotune, inputs, lbm

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    _ensure_built()
    torch.cuda.set_device(0)

    nx, nr = 2048, 512
    p, inlet, _ = inputs.workload_single(n_t=20000)
    nodes = nx * nr
    shape = autotune.best_shape(p, inlet, "fp32")
    info = lbm.tile_shape_info(shape)
    wall, ms_step, _ = time_jet(p, inlet, "fp32", args.steps, args.warmup, tile_shape=shape)
    glups = nodes * args.steps / wall / 1e9
    ms_launch = ms_step * info["steps"]
    updates_per_launch = nodes * info["steps"]
    alg_bytes = BYTES_PER_NODE["fp32"] * updates_per_launch
    achieved = alg_bytes / (ms_launch * 1e-3) / 1e9
    traffic = read_traffic(f"traffic_{kernel_of(info).split('_')[0]}_fp32_2048x512.txt")
    line = {
        "metric": "GLUPS & % HBM peak, FP32 vs FP16-storage; batched-jet p50/p99 solve latency",
        "value": round(glups, 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single axisymmetric jet, 2048 axial x 512 radial nodes, FP32 "
                               "populations, parabolic inlet R=32 U_max=0.08 with 1% noise, "
                               "T_in=1, C_s=0.17, tau=0.6, property tables seed 1",
                   "nx": nx, "nr": nr, "precision": "fp32", "graph_steps": 50,
                   "tile_shape": info},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kernel_of(info),
                     "steps_per_launch": info["steps"],
                     "node_updates_per_launch": updates_per_launch,
                     "bytes_per_node_update": BYTES_PER_NODE["fp32"],
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_ms_per_launch": round(ms_launch, 5),
                     "dram_GBps": (round(traffic / (ms_launch * 1e-3) / 1e9, 1)
                                   if traffic else None),
                     "alu": alu_roofline(kernel_of(info), nodes, ms_step)},
    }
    if not args.no_extra:
        extra = {}
        steps_x = max(200, args.steps // 4)

        def entry(prec, q, w, ms, n_nodes, n_steps):
            # ms: per step; algorithmic bytes per node update over the step time
            inf = lbm.tile_shape_info(q)
            return {"glups": round(n_nodes * n_steps / w / 1e9, 3), "tile_shape": inf,
                    "hbm_frac": round(BYTES_PER_NODE[prec] * n_nodes /
                                      (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

        # the same jet with one step per launch (the best one-step shape)
        q1 = autotune.best_shape(p, inlet, "fp32", steps=1)
        w, ms, _ = time_jet(p, inlet, "fp32", steps_x, args.warmup // 2, tile_shape=q1)
        extra["fp32_2048x512_one_step"] = entry("fp32", q1, w, ms, nodes, steps_x)
        for prec in ("fp16", "bf16", "fp16sr"):
            q = autotune.best_shape(p, inlet, prec)
            w, ms, _ = time_jet(p, inlet, prec, steps_x, args.warmup // 2, tile_shape=q)
            extra[f"{prec}_2048x512"] = entry(prec, q, w, ms, nodes, steps_x)
        pl, inl, _ = inputs.workload_large(n_t=4000)
        nodes_l = pl["nx"] * pl["nr"]
        steps_l = max(100, args.steps // 10)
        for prec in ("fp32", "fp16", "fp16sr"):
            q = autotune.best_shape(pl, inl, prec)
            w, ms, _ = time_jet(pl, inl, prec, steps_l, 100, tile_shape=q)
            extra[f"{prec}_4096x1024"] = entry(prec, q, w, ms, nodes_l, steps_l)
        # one buffer updated in place (half the memory, one step per launch)
        for tag, (pp, ii, nn, ss) in (("2048x512", (p, inlet, nodes, steps_x)),
                                      ("4096x1024", (pl, inl, nodes_l, steps_l))):
            w, ms, _ = time_jet(pp, ii, "fp32", ss, 100, layout="single")
            extra[f"fp32_{tag}_single_buffer"] = {
                "glups": round(nn * ss / w / 1e9, 3),
                "bytes": lbm.bytes_required(pp, "fp32", "single"),
                "two_buffer_bytes": lbm.bytes_required(pp, "fp32", "two"),
                "hbm_frac": round(BYTES_PER_NODE["fp32"] * nn / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        # practical streaming ceiling: a plain copy of each jet's two-buffer footprint
        extra["copy_kernel"] = {tag: copy_ceiling(lbm.bytes_required(pp, "fp32", "two") // 2)
                                for tag, pp in (("2048x512_fp32", p), ("4096x1024_fp32", pl))}
        extra["batch_64_jets"] = bench_batch()
        extra["serving_fp16"] = bench_serving(precision="fp16")
        extra["serving_fp32"] = bench_serving(precision="fp32")
        line["extra"] = extra
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, inlet)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
