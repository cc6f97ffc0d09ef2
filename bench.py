"""Benchmark of the axisymmetric D2Q9 + D2Q4 LBGK-LES step on one MI355X.

A step is one time step of the whole hot path over the 2048 x 512 jet: edge
pulls, moments, properties, Smagorinsky relaxation time, sources, collision
and store, plus the FP64 conservation check once per 1000 steps.  The steps
are replayed from HIP graphs captured before the warm-up, or, for timed
regions under 200 steps, launched directly as the same groups.  The timed
region (`--steps`, bracketed by device syncs) runs the check after every full
1000 steps; a remainder of r steps is charged r/1000 of the check's measured
cost.
Throughput (`value`) is GLUPS, lattice node updates per second / 1e9, from
that wall clock.

`roofline`: HBM bandwidth at the algorithmic 104 B per node update for FP32
storage (13 populations read and written) and 52 B for 16-bit storage.
`achieved` = those bytes times the node updates of one launch, divided by
the launch duration, from HIP events on the solver's stream around the step
launches of the timed region (`event_us_per_launch`).  The average duration
of the same kernel in the committed rocprofv3 summary is given beside it
(`rocprof_us_per_launch`).  A two-step launch updates each node twice while
reading and writing each population once; `traffic` is the HBM bytes one
launch moves by the rocprofv3 counters (committed summary), and
`traffic_GBps` their rate.

Prints one JSON line.  Extras: one step per launch, FP16 / BF16 / FP16SR
storage on the same jet, the 4096 x 1024 jet (a working set above the
256 MB Infinity Cache), the single-buffer layout, a plain copy's ceiling,
the 64-jet batch against looped single-jet runs, the serving workload, and
the FP64 oracle timed on the host cores on a bounded sample.
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
CODEC = {"fp32": "CodecF32", "fp16": "CodecF16", "bf16": "CodecBF16", "fp16sr": "CodecF16SR"}
# Vector ALU issue: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz (a wave64 FP32
# instruction every 4 cycles per SIMD; packed FP32 not used), lane-ops/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions in the collision of one FP32 node update as compiled for
# gfx950 (eqs. 2-6 and 1 from the pulled values to the relaxed ones): the
# static count of a kernel that loads a node's 13 values, collides and stores
# them, less that of the same kernel without the collision.  The counters'
# executed figure per kernel is read from profiles/valu_*.txt.
VALU_COLLISION = 166


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _ensure_built():
    from paper_1002_3028_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def kernel_of(info):
    return "pair_kernel" if info["steps"] == 2 else "step_kernel"


def _summary(name):
    """key -> value of a committed summary under profiles/, or None when absent
    or taken on another version of the kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#") and "|" not in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    from paper_1002_3028_amd.profsum import kernel_source_sha256
    if vals.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return vals


def read_summary(name, key):
    vals = _summary(name)
    try:
        return float(vals[key]) if vals else None
    except (KeyError, ValueError):
        return None


def read_traffic(name):
    """Per-launch HBM bytes (read + write) from a committed counter summary."""
    return read_summary(name, "hbm_bytes_per_launch")


def read_trace_us(name, kernel):
    """Average duration (us) of the kernel whose name contains `kernel` in a
    committed rocprofv3 --stats summary, when taken on the current source."""
    if _summary(name) is None:
        return None
    for line in open(os.path.join(ROOT, "profiles", name)):
        cols = [c.strip() for c in line.split("|")]
        if len(cols) == 6 and kernel in cols[0]:
            return float(cols[2])
    return None


def alu_roofline(kernel, prec, tag, nodes, ms_step):
    """The launch against vector-ALU issue: VALU instructions executed per
    node update (SQ_INSTS_VALU over node updates / 64, from the committed
    counter summary of this kernel; null when stale) x node updates per
    second."""
    kind = kernel.split("_")[0]
    executed = read_summary(f"valu_{kind}_{prec}_{tag}.txt", "valu_per_node_update")
    out = {"unit": "T lane-op/s", "peak": round(VALU_PEAK_TOPS, 2),
           "valu_collision_per_node_update": VALU_COLLISION,
           "valu_executed_per_node_update": executed, "achieved": None, "frac": None}
    if executed:
        achieved = executed * nodes / (ms_step * 1e-3) / 1e12
        out.update(achieved=round(achieved, 2), frac=round(achieved / VALU_PEAK_TOPS, 4))
    return out


def graph_group(steps, cap=50):
    """Steps per captured graph: the largest even count <= cap that divides
    `steps`, so that every timed step is a graph replay (cap if none)."""
    for g in range(min(cap, steps) // 2 * 2, 1, -2):
        if steps % g == 0:
            return g
    return cap


def time_jet(params, inlet, precision, steps, warmup, check_every=1000, tile_shape=None,
             layout="two"):
    """Time `steps` steps of one jet, the FP64 conservation check included at
    its cadence (once per `check_every` steps).

    Launches: for 200 steps or more, HIP graphs of graph_group(steps) steps,
    captured (and replayed once, dry) when the solver is set up; for shorter
    timed regions, directly launched groups (the same launches, offset from
    the descriptor, with no advance kernel), which start the device on the
    first kernel instead of after the whole graph has been submitted.  The
    warm-up runs right before the timed region, which is bracketed by device
    syncs.  The check runs inside it after every full `check_every` steps; a
    remainder of r steps is charged r / check_every of the check's cost,
    measured after the region (median of three).  Returns a dict:
    wall seconds (charge included), the charge, GPU milliseconds per step from
    HIP events on the solver's stream around the step launches only, and the
    launch mode."""
    import torch
    from paper_1002_3028_amd import lbm

    g = graph_group(steps) if steps >= 200 else 0
    with lbm.Solver(params, precision, graph_steps=g, tile_shape=tile_shape,
                    layout=layout) as s:
        s.set_inlet(*inlet)
        if steps >= check_every:
            s.conservation()  # (its first call sets up the reduction's buffers)
        # the timing events, one pair per window between checks, exist before
        # the clock starts (a first record creates the device event, a host
        # call of several microseconds)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(-(-steps // check_every))]
        for e0, e1 in evs:
            e0.record(s.torch_stream)
            e1.record(s.torch_stream)
        s.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        for e0, e1 in evs:
            n = min(check_every, steps - done)
            e0.record(s.torch_stream)
            s.step(n)
            e1.record(s.torch_stream)
            done += n
            if n == check_every:
                s.conservation()  # FP64 reduction + stability check (syncs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.sync()  # the solver's own stability flag, read outside the clock
        ev_ms = sum(a.elapsed_time(b) for a, b in evs)
        costs = []
        for _ in range(3):
            t = time.perf_counter()
            s.conservation()
            costs.append(time.perf_counter() - t)
        check_s = sorted(costs)[1]
    charge = (steps % check_every) / check_every * check_s
    return {"wall_s": wall + charge, "check_charge_s": charge, "check_s": check_s,
            "event_ms_per_step": ev_ms / steps,
            "launch": f"graphs of {g} steps" if g else "direct groups"}


def roofline_block(prec, info, nodes, ms_step, traffic_name, trace_name=None, tag=None):
    """HBM roofline of the dominant kernel: algorithmic bytes per launch over
    the launch duration from HIP events (steps only, graph replays)."""
    kernel = kernel_of(info)
    ms_launch = ms_step * info["steps"]
    updates = nodes * info["steps"]
    alg = BYTES_PER_NODE[prec] * updates
    achieved = alg / (ms_launch * 1e-3) / 1e9
    traffic = read_traffic(traffic_name) if traffic_name else None
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kernel,
           "steps_per_launch": info["steps"], "node_updates_per_launch": updates,
           "bytes_per_node_update": BYTES_PER_NODE[prec],
           "algorithmic_bytes_per_launch": alg,
           "event_us_per_launch": round(ms_launch * 1e3, 3),
           "rocprof_us_per_launch": (read_trace_us(trace_name, f"{kernel}<lbmx::{CODEC[prec]}")
                                     if trace_name else None),
           "traffic_GBps": (round(traffic / (ms_launch * 1e-3) / 1e9, 1) if traffic else None)}
    if tag:
        out["alu"] = alu_roofline(kernel, prec, tag, nodes, ms_step)
    return out


def bench_batch(n_jets=64, steps=5000, precision="fp32", looped=True):
    """64 jets of uneven sizes (seed 2) advanced together, one persistent
    launch per step (or pair of steps) per cohort, with the launch
    configuration the batch tuner picks for this set (tile shape, grid,
    cohort size, streams; tuned once and cached) and, for comparison, with
    the batch's defaults; with `looped`, against the same jets run one after
    another through the single-jet path.  Aggregate GLUPS of each."""
    import torch
    from paper_1002_3028_amd import autotune, inputs, lbm

    jets = inputs.batch_jets(n_jets, seed=2, steps=steps)
    nodes = sum(p["nx"] * p["nr"] for p, _, _ in jets)
    budget = sum(lbm.bytes_required(p, precision) for p, _, _ in jets) + (64 << 20)
    tuned = autotune.tune_batch([(p, inlet) for p, inlet, _ in jets], precision)
    groups = steps // 50

    def batched(cfg):
        with lbm.Batch(budget, n_jets, precision) as b:
            if cfg is not None:
                autotune.apply_batch(b, cfg)
            for p, inlet, _ in jets:
                b.admit(p, inlet, steps + 100)
            b.run(50)
            b.sync()
            t0 = time.perf_counter()
            for _ in range(groups):
                b.run(50)
            b.sync()
            return nodes * groups * 50 / (time.perf_counter() - t0) / 1e9

    out = {"jets": n_jets, "nodes": nodes, "steps": groups * 50, "precision": precision,
           "tuned": {k: tuned[k] for k in ("shape", "workgroups", "cohort_mib", "streams")},
           "tuned_shape": lbm.tile_shape_info(tuned["shape"]),
           "batched_glups": round(batched(tuned), 3),
           "batched_default_glups": round(batched(None), 3)}
    if not looped:
        return out
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
    out["looped_single_glups"] = round(nodes * steps / t_loop / 1e9, 3)
    return out


def bench_serving(n_requests=2000):
    """The serving workload (Poisson trace of seed 3): saturated capacity of
    FP32 and FP16 storage (every request admitted at once), then the same
    trace at one arrival rate, 0.7 x the FP32 capacity: p50/p99 latency
    (arrival to completion) and throughput.  FP16 as served by default
    stores requests longer than the FP16 step limit (every request: the limit
    is 0) with stochastic rounding (serve.route); "fp16_unrouted" keeps every
    request in FP16 rounded to nearest."""
    from paper_1002_3028_amd import inputs, serve

    out = {"requests": n_requests, "trace_seed": 3,
           "fp16_step_limit": serve.FP16_STEP_LIMIT}
    cap = {}
    for prec in ("fp32", "fp16"):
        log(f"serving {prec}: capacity, {n_requests} requests")
        c, _ = serve.serve(inputs.arrival_trace(n_requests, 3, rate=1.0), prec,
                           16 << 30, 256, 100, realtime=False)
        cap[prec] = c
        out[f"{prec}_capacity_req_per_s"] = c["requests_per_s"]
        out[f"{prec}_capacity_glups"] = c["glups"]
    out["fp16_storage_counts"] = cap["fp16"]["storage_counts"]
    rate = 0.7 * cap["fp32"]["requests_per_s"]
    out["rate_req_per_s"] = round(rate, 3)
    trace = inputs.arrival_trace(n_requests, 3, rate=rate)
    for name, prec, long_after in (("fp32", "fp32", -1), ("fp16", "fp16", serve.FP16_STEP_LIMIT),
                                   ("fp16_unrouted", "fp16", -1)):
        log(f"serving {name}: {rate:.1f} requests/s")
        run, _ = serve.serve(trace, prec, 16 << 30, 256, 100, realtime=True,
                             long_after=long_after)
        out[name] = {"p50_s": run["p50_s"], "p99_s": run["p99_s"], "mean_s": run["mean_s"],
                     "served_req_per_s": run["requests_per_s"], "glups": run["glups"],
                     "peak_slots": run["peak_slots"],
                     # share of the loop's wall time in which the device ran a group
                     "device_busy": run["device_busy"]}
    return out


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


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next((ln.split(":", 1)[1].strip() for ln in fh
                         if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(params, inlet, budget_s=12.0):
    """The FP64 oracle as it stands on the host cores (OpenMP over radial
    rows), on a bounded sample of the same jet: the steps that fit about
    budget_s after two warm steps."""
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
                      f"(FP64, OpenMP over radial rows), {dt:.1f} s",
            "cpu": _cpu_model(), "compiler": "gcc -O2 -std=c11 -ffp-contract=off -fopenmp"}


def oracle_timing():
    """The FP64 oracle on one thread and on every host core (OpenMP over radial
    rows; bit-identical results for any thread count): the 128 x 32 jet for
    its 500 steps, the first 200 steps of the 2048 x 512 jet and 100 steps of
    the 1024 x 256 twin of the 4096 x 1024 jet, warm (after two steps), median
    of three for runs under a second."""
    import platform
    import oracle
    from paper_1002_3028_amd import inputs

    model = _cpu_model()
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
    ap.add_argument("--batch-steps", type=int, default=5000,
                    help="steps of the 64-jet batch leg")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the serving leg")
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
    log(f"headline: 2048x512 fp32, shape {shape}, {args.steps} steps")
    t = time_jet(p, inlet, "fp32", args.steps, args.warmup, tile_shape=shape)
    glups = nodes * args.steps / t["wall_s"] / 1e9
    line = {
        "metric": "GLUPS & % HBM peak, FP32 vs FP16-storage; batched-jet p50/p99 solve latency",
        "value": round(glups, 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t["wall_s"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single axisymmetric jet, 2048 axial x 512 radial nodes, FP32 "
                               "populations, parabolic inlet R=32 U_max=0.08 with 1% noise, "
                               "T_in=1, C_s=0.17, tau=0.6, property tables seed 1",
                   "nx": nx, "nr": nr, "precision": "fp32", "launch": t["launch"],
                   "fp64_check_every": 1000,
                   "fp64_check_charged_s": round(t["check_charge_s"], 7),
                   "tile_shape": info},
        # the committed trace of the same launch mode: the 20-step region of
        # direct launches, or the last 1 000 launches of a 2 000-step run
        "roofline": roofline_block("fp32", info, nodes, t["event_ms_per_step"],
                                   f"traffic_{kernel_of(info).split('_')[0]}_fp32_2048x512.txt",
                                   "pair_kernel_fp32_2048x512_20steps_kernel_trace.txt"
                                   if t["launch"] == "direct groups"
                                   else "pair_kernel_fp32_2048x512_kernel_trace.txt",
                                   tag="2048x512"),
    }
    if not args.no_extra:
        extra = {}
        steps_x = max(200, args.steps // 4)
        warm_x = max(10, args.warmup // 2)

        def entry(prec, q, t, n_nodes, n_steps, traffic_name=None, trace_name=None):
            inf = lbm.tile_shape_info(q)
            e = {"glups": round(n_nodes * n_steps / t["wall_s"] / 1e9, 3), "tile_shape": inf,
                 "event_glups": round(n_nodes / (t["event_ms_per_step"] * 1e-3) / 1e9, 3)}
            e["roofline"] = roofline_block(prec, inf, n_nodes, t["event_ms_per_step"],
                                           traffic_name, trace_name)
            return e

        # the same jet with one step per launch (the best one-step shape)
        q1 = autotune.best_shape(p, inlet, "fp32", steps=1)
        tt = time_jet(p, inlet, "fp32", steps_x, warm_x, tile_shape=q1)
        extra["fp32_2048x512_one_step"] = entry("fp32", q1, tt, nodes, steps_x,
                                                "traffic_step_fp32_2048x512.txt")
        for prec in ("fp16", "bf16", "fp16sr"):
            q = autotune.best_shape(p, inlet, prec)
            log(f"2048x512 {prec}, shape {q}")
            tt = time_jet(p, inlet, prec, steps_x, warm_x, tile_shape=q)
            kind = kernel_of(lbm.tile_shape_info(q)).split("_")[0]
            extra[f"{prec}_2048x512"] = entry(prec, q, tt, nodes, steps_x,
                                              f"traffic_{kind}_{prec}_2048x512.txt")
        # the 4096 x 1024 jet: its FP32 buffers (436 MB) exceed the Infinity
        # Cache, so this is the HBM-bandwidth case
        pl, inl, _ = inputs.workload_large(n_t=4000)
        nodes_l = pl["nx"] * pl["nr"]
        steps_l = max(100, args.steps // 10)
        for prec in ("fp32", "fp16", "fp16sr"):
            q = autotune.best_shape(pl, inl, prec)
            log(f"4096x1024 {prec}, shape {q}")
            tt = time_jet(pl, inl, prec, steps_l, warm_x, tile_shape=q)
            kind = kernel_of(lbm.tile_shape_info(q)).split("_")[0]
            extra[f"{prec}_4096x1024"] = entry(prec, q, tt, nodes_l, steps_l,
                                               f"traffic_{kind}_{prec}_4096x1024.txt",
                                               f"{kind}_kernel_{prec}_4096x1024_kernel_trace.txt")
        # one buffer updated in place (half the memory, one step per launch)
        for tag, (pp, ii, nn, ss) in (("2048x512", (p, inlet, nodes, steps_x)),
                                      ("4096x1024", (pl, inl, nodes_l, steps_l))):
            tt = time_jet(pp, ii, "fp32", ss, warm_x, layout="single")
            extra[f"fp32_{tag}_single_buffer"] = {
                "glups": round(nn * ss / tt["wall_s"] / 1e9, 3),
                "bytes": lbm.bytes_required(pp, "fp32", "single"),
                "two_buffer_bytes": lbm.bytes_required(pp, "fp32", "two"),
                "hbm_frac": round(BYTES_PER_NODE["fp32"] * nn / (tt["event_ms_per_step"] * 1e-3)
                                  / 1e9 / HBM_PEAK_GBS, 4)}
        # practical streaming ceiling: a plain copy of each jet's two-buffer footprint
        extra["copy_kernel"] = {tag: copy_ceiling(lbm.bytes_required(pp, "fp32", "two") // 2)
                                for tag, pp in (("2048x512_fp32", p), ("4096x1024_fp32", pl))}
        log("64-jet batch")
        extra["batch_64_jets"] = bench_batch(steps=args.batch_steps)
        log("64-jet batch, FP16 storage")
        extra["batch_64_jets_fp16"] = bench_batch(steps=args.batch_steps, precision="fp16",
                                                  looped=False)
        log("serving")
        extra["serving"] = bench_serving(args.serving_requests)
        line["extra"] = extra
    if not args.no_cpu:
        log("oracle on the host cores")
        line["cpu_baseline"] = cpu_baseline(p, inlet)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
