"""The counter summaries that bench.py reads: traffic and VALU figures from
synthetic rocprofv3 CSVs, and the source check that turns a summary taken on
other kernel sources into null."""
import csv
import os

import pytest

HEADER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEADER)
        for q, (kernel, counter, value) in enumerate(rows):
            w.writerow([q, kernel, counter, value])
    return str(path)


def _run(args):
    import sys
    from paper_1002_3028_amd import profsum
    old = sys.argv
    sys.argv = ["profsum"] + args
    try:
        profsum.main()
    finally:
        sys.argv = old


def _vals(path):
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def test_traffic_scales_by_the_copy(tmp_path):
    """FETCH reads half and WRITE all of a 256 MiB copy here: a kernel whose
    counters read 50 and 100 KiB moves 100 + 100 KiB."""
    mib = 256 * 1024  # KiB
    fetch = _csv(tmp_path / "f.csv", [("copy_kernel(x)", "FETCH_SIZE", mib / 2),
                                      ("pair_kernel<a>", "FETCH_SIZE", 50.0),
                                      ("pair_kernel<a>", "FETCH_SIZE", 50.0)])
    write = _csv(tmp_path / "w.csv", [("copy_kernel(x)", "WRITE_SIZE", mib),
                                      ("pair_kernel<a>", "WRITE_SIZE", 100.0)])
    out = tmp_path / "t.txt"
    _run(["traffic", "--fetch", fetch, "--write", write, "--kernel", "pair_kernel",
          "--nodes", "10", "--bytes-per-node", "40", "--out", str(out), "--title", "t",
          "--command-fetch", "cf", "--command-write", "cw"])
    v = _vals(out)
    assert float(v["fetch_factor"]) == pytest.approx(0.5)
    assert float(v["hbm_bytes_per_launch"]) == pytest.approx(200 * 1024)
    assert float(v["traffic_over_algorithmic"]) == pytest.approx(200 * 1024 / 400, rel=1e-4)


def test_valu_per_update(tmp_path):
    """6400 instructions issued by the two waves that cover 128 node updates
    (64 lanes each): 6400 / (128 / 64) = 3200 per node update."""
    rows = [("step_kernel<b>", "SQ_INSTS_VALU", 6400.0), ("step_kernel<b>", "SQ_WAVES", 2.0)]
    out = tmp_path / "v.txt"
    _run(["valu", "--csv", _csv(tmp_path / "v.csv", rows), "--kernel", "step_kernel",
          "--updates", "128", "--out", str(out), "--title", "t", "--command", "c"])
    v = _vals(out)
    assert float(v["valu_per_wave"]) == pytest.approx(3200.0)
    assert float(v["valu_per_node_update"]) == pytest.approx(3200.0)


def test_bench_reads_only_current_summaries(tmp_path, monkeypatch):
    import bench
    from paper_1002_3028_amd.profsum import kernel_source_sha256
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.txt").write_text(f"hbm_bytes_per_launch: 123\nkernel_source_sha256: "
                                f"{kernel_source_sha256()}\n")
    (prof / "y.txt").write_text("hbm_bytes_per_launch: 456\nkernel_source_sha256: 0\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("x.txt") == 123.0
    assert bench.read_traffic("y.txt") is None
    assert bench.read_traffic("missing.txt") is None


def test_bench_reads_kernel_average_from_stats(tmp_path, monkeypatch):
    """A --stats summary written by profsum gives bench.py the average
    duration of the named kernel, and nothing once the sources change."""
    import bench
    rows = [{"Name": "void lbmx::pair_kernel<lbmx::CodecF32, 8, 4, 5, 8>(x)", "Calls": "10",
             "AverageNs": "27263.0", "MinNs": "26000", "MaxNs": "28000", "Percentage": "90"},
            {"Name": "lbmx::advance_kernel(x)", "Calls": "1", "AverageNs": "1500.0",
             "MinNs": "1500", "MaxNs": "1500", "Percentage": "10"}]
    path = tmp_path / "s.csv"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    prof = tmp_path / "profiles"
    prof.mkdir()
    _run(["stats", "--csv", str(path), "--out", str(prof / "k.txt"), "--title", "t",
          "--command", "c"])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_trace_us("k.txt", "pair_kernel<lbmx::CodecF32") == pytest.approx(27.263)
    assert bench.read_trace_us("k.txt", "pair_kernel<lbmx::CodecF16") is None
    text = (prof / "k.txt").read_text().replace("kernel_source_sha256: ", "kernel_source_sha256: 0")
    (prof / "k.txt").write_text(text)
    assert bench.read_trace_us("k.txt", "pair_kernel<lbmx::CodecF32") is None


@pytest.mark.parametrize("steps,group", [(20, 20), (20000, 50), (2000, 50), (200, 50),
                                         (30, 30), (42, 42), (5, 50), (98, 14)])
def test_bench_graph_group_divides_the_timed_steps(steps, group):
    """Every timed step is a replay of the graph captured before the clock
    starts: the group is the largest even divisor up to 50."""
    import bench
    g = bench.graph_group(steps)
    assert g == group
    assert g % 2 == 0 and (steps % g == 0 or g == 50)


def test_busy_counts_overlapping_kernels_once(tmp_path):
    """Two streams' kernels overlap: the busy time is the union of the
    intervals, and only the idle stretch between them is a gap."""
    rows = [("KERNEL_DISPATCH", 0, 100), ("KERNEL_DISPATCH", 50, 150),   # overlap
            ("KERNEL_DISPATCH", 150, 200),                                # touching
            ("KERNEL_DISPATCH", 60_200, 60_300)]                          # after a 60 us gap
    path = tmp_path / "k.csv"
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Start_Timestamp", "End_Timestamp"])
        w.writerows(rows)
    out = tmp_path / "b.txt"
    _run(["busy", "--csv", str(path), "--gap-us", "20", "--out", str(out), "--title", "t",
          "--command", "c"])
    v = _vals(out)
    assert float(v["busy_fraction"]) == pytest.approx(300 / 60_300, abs=1e-4)
    assert int(v["gaps_over_20.0us"]) == 1
    assert float(v["largest_gap_us"]) == pytest.approx(60.0)


def test_stats_window_of_a_trace(tmp_path, monkeypatch):
    """stats --trace tabulates only the tail that starts at the first of the
    kernel's last N dispatches: the tuning launches before it (and their
    short dry runs) stay out of the average bench.py compares with."""
    rows = [("tune_kernel", 0, 5), ("pair_kernel", 10, 12),        # a dry replay
            ("pair_kernel", 20, 40), ("pair_kernel", 50, 70),
            ("advance_kernel", 70, 74), ("pair_kernel", 80, 110)]
    path = tmp_path / "t.csv"
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerows([("KERNEL_DISPATCH",) + r for r in rows])
    out = tmp_path / "s.txt"
    _run(["stats", "--trace", str(path), "--kernel", "pair_kernel", "--last", "3",
          "--out", str(out), "--title", "t", "--command", "c"])
    from paper_1002_3028_amd import profsum
    lines = [ln.split("|") for ln in open(out) if ln.count("|") == 5 and not ln.startswith("#")]
    table = {c[0].strip(): [x.strip() for x in c[1:]] for c in lines}
    assert set(table) == {"pair_kernel", "advance_kernel"}
    assert table["pair_kernel"][0] == "3"
    assert float(table["pair_kernel"][1]) == pytest.approx(70 / 3 / 1e3, abs=1e-3)
    assert float(table["advance_kernel"][1]) == pytest.approx(0.004)
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles", exist_ok=True)
    os.replace(out, tmp_path / "profiles" / "s.txt")
    assert bench.read_trace_us("s.txt", "pair_kernel") == pytest.approx(0.023, abs=1e-3)
    assert profsum.kernel_source_sha256() in open(tmp_path / "profiles" / "s.txt").read()
