"""Summaries of rocprofv3 output for the repository's profiles/ folder.

  stats:   per-kernel duration table from a --kernel-trace --stats run
  traffic: HBM bytes per launch of one kernel from two --pmc runs
           (FETCH_SIZE, WRITE_SIZE), each scaled by what the same counter
           reads for the probe's copy of known size.
  valu:    vector-ALU instructions executed per node update from a --pmc
           run of SQ_INSTS_VALU and SQ_WAVES (one instruction of a wave
           serves 64 lanes, so per update = total / (updates / 64)).
  busy:    from a --kernel-trace run, the share of the traced span in which
           some kernel runs (union of the dispatch intervals, so kernels on
           several streams count once) and the idle gaps between kernels.

Each writes a short text file that records the command which produced the
figures and the SHA-256 of the kernel sources they were taken on.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("lbm_device.hpp", "lbm_kernels.hpp")


def kernel_source_sha256() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _window_stats(trace_csv, kernel, last):
    """Per-kernel rows (as in a --stats table) over the tail of a kernel trace
    that starts with the first of the last `last` dispatches of `kernel`:
    the timed region of a run, without its set-up and tuning launches."""
    rows = [r for r in _rows(trace_csv) if r.get("Kind", "KERNEL_DISPATCH") == "KERNEL_DISPATCH"]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    mine = [q for q, r in enumerate(rows) if kernel in r["Kernel_Name"]]
    if len(mine) < last:
        raise SystemExit(f"{len(mine)} dispatches of {kernel!r}, fewer than {last}")
    per = {}
    for r in rows[mine[-last]:]:
        per.setdefault(r["Kernel_Name"], []).append(
            int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in per.values())
    out = [{"Name": k, "Calls": len(v), "AverageNs": sum(v) / len(v), "MinNs": min(v),
            "MaxNs": max(v), "Percentage": 100.0 * sum(v) / total} for k, v in per.items()]
    return sorted(out, key=lambda r: -r["Percentage"])


def stats(args):
    if args.trace:
        rows = _window_stats(args.trace, args.kernel, args.last)
    else:
        rows = _rows(args.csv)
    lines = [f"# rocprofv3 kernel statistics: {args.title}",
             f"# command: {args.command}"]
    if args.trace:
        lines.append(f"# from the kernel trace, over the last {args.last} dispatches of "
                     f"{args.kernel} and everything after the first of them")
    lines.append("# kernel | calls | average us | min us | max us | share %")
    for r in rows[: args.top]:
        name = r["Name"]
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"{name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.3f} | "
                     f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | "
                     f"{float(r['Percentage']):.2f}")
    lines.append(f"kernel_source_sha256: {kernel_source_sha256()}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    out = {}
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(args):
    fetch = _per_kernel(args.fetch, "FETCH_SIZE")
    write = _per_kernel(args.write, "WRITE_SIZE")

    def pick(d, key):
        hits = [v for k, v in d.items() if key in k]
        if not hits:
            raise SystemExit(f"no dispatch of a kernel matching {key!r}")
        return [x for v in hits for x in v]

    copy_bytes = args.copy_mib * (1 << 20)
    f_copy = statistics.median(pick(fetch, "copy_kernel")) * 1024
    w_copy = statistics.median(pick(write, "copy_kernel")) * 1024
    f_factor, w_factor = f_copy / copy_bytes, w_copy / copy_bytes
    # launches of unequal size (the cohorts of a batch) take the mean
    avg = statistics.mean if args.mean else statistics.median
    f_k = avg(pick(fetch, args.kernel)) * 1024 / f_factor
    w_k = avg(pick(write, args.kernel)) * 1024 / w_factor
    alg = args.bytes_per_node * args.nodes
    lines = [
        f"# HBM traffic per launch of {args.kernel} ({args.title})",
        f"# command (fetch): {args.command_fetch}",
        f"# command (write): {args.command_write}",
        f"copy_calibration_bytes: {copy_bytes}",
        f"fetch_factor: {f_factor:.5f}",
        f"write_factor: {w_factor:.5f}",
        f"fetch_bytes_per_launch: {f_k:.0f}",
        f"write_bytes_per_launch: {w_k:.0f}",
        f"hbm_bytes_per_launch: {f_k + w_k:.0f}",
        f"algorithmic_bytes_per_launch: {alg}",
        f"traffic_over_algorithmic: {(f_k + w_k) / alg:.4f}",
        f"kernel_source_sha256: {kernel_source_sha256()}",
    ]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def valu(args):
    insts = [x for k, v in _per_kernel(args.csv, "SQ_INSTS_VALU").items() if args.kernel in k
             for x in v]
    waves = [x for k, v in _per_kernel(args.csv, "SQ_WAVES").items() if args.kernel in k
             for x in v]
    if not insts or not waves:
        raise SystemExit(f"no SQ_INSTS_VALU / SQ_WAVES for a kernel matching {args.kernel!r}")
    per_launch = statistics.median(insts)
    lines = [
        f"# vector-ALU instructions of {args.kernel} ({args.title})",
        f"# command: {args.command}",
        f"launches: {len(insts)}",
        f"valu_instructions_per_launch: {per_launch:.0f}",
        f"waves_per_launch: {statistics.median(waves):.0f}",
        f"valu_per_wave: {per_launch / statistics.median(waves):.1f}",
        f"node_updates_per_launch: {args.updates}",
        f"valu_per_node_update: {per_launch / (args.updates / 64):.1f}",
    ]
    # wave-state counters, when the same pass collected them (per launch,
    # medians): where a wave's life goes
    extra = {}
    for c in ("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
              "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS"):
        v = [x for k, vs in _per_kernel(args.csv, c).items() if args.kernel in k for x in vs]
        if v:
            extra[c] = statistics.median(v)
            lines.append(f"{c.lower()}_per_launch: {extra[c]:.0f}")
    if "SQ_WAVE_CYCLES" in extra:
        wc = extra["SQ_WAVE_CYCLES"]
        if "SQ_ACTIVE_INST_VALU" in extra:
            lines.append(f"valu_issue_share_of_wave_cycles: {extra['SQ_ACTIVE_INST_VALU'] / wc:.3f}")
        if "SQ_WAIT_INST_ANY" in extra:
            lines.append(f"waiting_share_of_wave_cycles: {extra['SQ_WAIT_INST_ANY'] / wc:.3f}")
        if "SQ_BUSY_CYCLES" in extra:
            lines.append(f"mean_waves_in_flight_per_busy_cycle: {wc / extra['SQ_BUSY_CYCLES']:.1f}")
    lines.append(f"kernel_source_sha256: {kernel_source_sha256()}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def busy(args):
    rows = [r for r in _rows(args.csv) if r.get("Kind", "KERNEL_DISPATCH") == "KERNEL_DISPATCH"]
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows)
    if args.skip:
        iv = iv[args.skip:]
    merged = []
    for a, b in iv:
        if merged and a <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], b)
        else:
            merged.append([a, b])
    span = merged[-1][1] - merged[0][0]
    run = sum(b - a for a, b in merged)
    gaps = sorted(merged[q + 1][0] - merged[q][1] for q in range(len(merged) - 1))
    big = [g for g in gaps if g > args.gap_us * 1000]
    lines = [f"# GPU busy time from a kernel trace: {args.title}",
             f"# command: {args.command}",
             f"dispatches: {len(iv)}",
             f"span_ms: {span / 1e6:.3f}",
             f"busy_fraction: {run / span:.4f}",
             f"gaps_over_{args.gap_us}us: {len(big)}",
             f"idle_in_those_gaps_ms: {sum(big) / 1e6:.3f}",
             f"median_gap_us: {statistics.median(gaps) / 1e3 if gaps else 0.0:.2f}",
             f"largest_gap_us: {gaps[-1] / 1e3 if gaps else 0.0:.1f}",
             f"kernel_source_sha256: {kernel_source_sha256()}"]
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("--csv", help="kernel_stats.csv")
    a.add_argument("--trace", help="kernel_trace.csv: tabulate a window of it instead")
    a.add_argument("--kernel", help="with --trace: substring of the timed kernel's name")
    a.add_argument("--last", type=int, default=0,
                   help="with --trace: the timed kernel's dispatches in the window")
    a.add_argument("--out", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--top", type=int, default=12)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True, help="substring of the kernel name")
    b.add_argument("--copy-mib", type=int, default=256)
    b.add_argument("--nodes", type=int, required=True)
    b.add_argument("--mean", action="store_true",
                   help="mean over launches (default: median)")
    b.add_argument("--bytes-per-node", type=int, required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--title", required=True)
    b.add_argument("--command-fetch", required=True)
    b.add_argument("--command-write", required=True)
    c = sub.add_parser("valu")
    c.add_argument("--csv", required=True)
    c.add_argument("--kernel", required=True, help="substring of the kernel name")
    c.add_argument("--updates", type=int, required=True, help="node updates per launch")
    c.add_argument("--out", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    d = sub.add_parser("busy")
    d.add_argument("--csv", required=True, help="kernel_trace.csv")
    d.add_argument("--gap-us", type=float, default=20.0)
    d.add_argument("--skip", type=int, default=0, help="leading dispatches to leave out")
    d.add_argument("--out", required=True)
    d.add_argument("--title", required=True)
    d.add_argument("--command", required=True)
    args = ap.parse_args()
    if args.cmd == "stats" and not (args.csv or (args.trace and args.kernel and args.last > 0)):
        ap.error("stats needs --csv, or --trace with --kernel and --last")
    {"stats": stats, "traffic": traffic, "valu": valu, "busy": busy}[args.cmd](args)


if __name__ == "__main__":
    main()
