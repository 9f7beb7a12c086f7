"""Profiling helpers: the launches that hardware counters are taken on, and
the text summaries made from rocprofv3's CSV output.

    # launches: a 1 GiB device copy (calibration), then outer-step updates
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o f -- \\
        python3 -m paper_1306_4161_amd.profiling launches --path fp64
    # summary file read back by bench.py (HBM bytes per launch)
    python3 -m paper_1306_4161_amd.profiling traffic --fetch OUT/f_counter_collection.csv \\
        --write OUT2/w_counter_collection.csv --kernel fp64_dma_kernel ...
    # MFMA-busy fraction and clock from a counter pass
    rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE --output-format csv -d OUT -o m -- \\
        python3 -m paper_1306_4161_amd.profiling launches --path fp64
    python3 -m paper_1306_4161_amd.profiling mfma OUT/m_counter_collection.csv --kernel fp64_dma_kernel ...
    # per-kernel time table from `rocprofv3 --kernel-trace --stats`
    python3 -m paper_1306_4161_amd.profiling stats OUT/kt_kernel_stats.csv --command "..."
    # the same over the steady state (first dispatches of each kernel left out)
    python3 -m paper_1306_4161_amd.profiling trace OUT/kt_kernel_trace.csv --skip 3 --command "..."

FETCH_SIZE and WRITE_SIZE count L2-to-memory traffic in KiB per dispatch.
Each is scaled by what it reads for a plain copy of known size (bytes copied
/ counted bytes), so that the figure is in true bytes.
"""
from __future__ import annotations

import argparse
import csv
import collections
import hashlib
import os
import shlex
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def code_only(text: str) -> str:
    """C++ source with its comments removed and white space collapsed (string
    and character literals kept as written)."""
    out = []
    i, n = 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(*names) -> str:
    """Hash of the code of the named csrc files: a profile summary records it,
    and bench.py uses a summary's counters only while the code is unchanged
    (edits to comments or layout do not count)."""
    h = hashlib.sha256()
    for nm in names:
        with open(os.path.join(ROOT, "paper_1306_4161_amd", "csrc", nm), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode("utf-8"))
    return h.hexdigest()[:16]


def launches(args):
    import torch
    from . import hsumma as hs
    from . import inputs
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    n = args.n
    if args.sigma > 0:
        A = inputs.exponent_spread(n, n, inputs.SEED_A, args.sigma)
        B = inputs.exponent_spread(n, n, inputs.SEED_B, args.sigma)
    else:
        A = inputs.uniform(n, n, inputs.SEED_A)
        B = inputs.uniform(n, n, inputs.SEED_B)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    del A, B
    dC = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    prec = {"fp64": hs.FP64, "bf16": hs.SPLIT_BF16, "int8": hs.SPLIT_INT8}[args.path]
    plan = hs.Plan(n, args.P, args.Q, args.G, args.b, args.M, prec=prec)
    ws = plan.workspace()
    for g in range(min(args.count, plan.num_outer_steps)):
        plan.outer_update(g, dA, dB, dC, ws=ws)
        torch.cuda.synchronize()
        print("launch %d done" % g, flush=True)


def _per_dispatch(path):
    """{dispatch id: (kernel name, {counter: summed value})}."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            did = int(r["Dispatch_Id"])
            name, vals = out.setdefault(did, (r["Kernel_Name"], collections.defaultdict(float)))
            vals[r["Counter_Name"]] += float(r["Counter_Value"])
    return out


def _mean(values):
    values = list(values)
    return sum(values) / len(values)


def traffic(args):
    fetch = _per_dispatch(args.fetch)
    write = _per_dispatch(args.write)

    def pick(table, counter, key):
        v = [vals[counter] for _, (nm, vals) in sorted(table.items()) if key in nm]
        if not v:
            raise SystemExit("no dispatch of %r with %s" % (key, counter))
        return v

    cf = _mean(pick(fetch, "FETCH_SIZE", COPY_KERNEL))
    cw = _mean(pick(write, "WRITE_SIZE", COPY_KERNEL))
    kf = pick(fetch, "FETCH_SIZE", args.kernel)
    kw = pick(write, "WRITE_SIZE", args.kernel)
    sf = COPY_BYTES / (cf * 1024.0)
    sw = COPY_BYTES / (cw * 1024.0)
    fb = _mean(kf) * 1024.0 * sf
    wb = _mean(kw) * 1024.0 * sw
    total = fb + wb
    lines = [
        "# HBM traffic per launch of %s, workload %s" % (args.kernel, args.workload),
        "# fetch command: %s" % args.fetch_command,
        "# write command: %s" % args.write_command,
        "# summary command: python3 -m paper_1306_4161_amd.profiling %s" % shlex.join(
            sys.argv[1:]),
        "# calibration: 1 GiB copy (%s) reads FETCH_SIZE %.1f KiB, WRITE_SIZE %.1f KiB"
        % (COPY_KERNEL, cf, cw),
        "kernel: %s" % args.kernel,
        "source_hash: %s" % source_hash(*args.source.split(",")),
        "dispatches: %d fetch, %d write" % (len(kf), len(kw)),
        "fetch_kib_raw_mean: %.1f" % _mean(kf),
        "write_kib_raw_mean: %.1f" % _mean(kw),
        "fetch_scale: %.4f" % sf,
        "write_scale: %.4f" % sw,
        "fetch_bytes_per_launch: %.6g" % fb,
        "write_bytes_per_launch: %.6g" % wb,
        "hbm_bytes_per_launch: %.6g" % total,
    ]
    if args.algorithmic:
        lines.append("algorithmic_bytes_per_launch: %.6g" % args.algorithmic)
        lines.append("traffic_over_algorithmic: %.3f" % (total / args.algorithmic))
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, end="")


def mfma(args):
    """MFMA-busy fraction and effective clock per dispatch of one kernel.

    GRBM_GUI_ACTIVE counts busy cycles of each XCD, summed over the XCDs;
    SQ_VALU_MFMA_BUSY_CYCLES counts cycles in which a SIMD's matrix core is
    busy, summed over every SIMD.  busy = MFMA cycles / (XCD cycles x SIMDs);
    clock = XCD cycles / dispatch duration.
    """
    rows = collections.defaultdict(lambda: collections.defaultdict(float))
    span = {}
    names = {}
    with open(args.csv) as f:
        for r in csv.DictReader(f):
            did = int(r["Dispatch_Id"])
            rows[did][r["Counter_Name"]] += float(r["Counter_Value"])
            span[did] = (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
            names[did] = r["Kernel_Name"]
    sel = [d for d in sorted(rows) if args.kernel in names[d]]
    if not sel:
        raise SystemExit("no dispatch of %r" % args.kernel)
    lines = ["# MFMA busy fraction and clock of %s, workload %s" % (args.kernel, args.workload),
             "# command: %s" % args.command,
             "# summary command: python3 -m paper_1306_4161_amd.profiling %s" % shlex.join(
                 sys.argv[1:]),
             "# busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / xcds x simds); "
             "clock = GRBM_GUI_ACTIVE / xcds / duration",
             "kernel: %s" % args.kernel,
             "source_hash: %s" % source_hash(*args.source.split(",")),
             "xcds: %d" % args.xcds, "simds: %d" % args.simds,
             "%-10s %12s %10s %10s" % ("dispatch", "duration_us", "clock_ghz", "mfma_busy")]
    busy_all, clk_all = [], []
    for d in sel:
        v = rows[d]
        cyc = v["GRBM_GUI_ACTIVE"] / args.xcds
        dur = (span[d][1] - span[d][0]) * 1e-9
        busy = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * args.simds)
        clk = cyc / dur / 1e9
        busy_all.append(busy)
        clk_all.append(clk)
        lines.append("%-10d %12.1f %10.3f %10.4f" % (d, dur * 1e6, clk, busy))
    lines.append("mean_mfma_busy: %.4f" % _mean(busy_all))
    lines.append("mean_clock_ghz: %.3f" % _mean(clk_all))
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, end="")


def stats(args):
    with open(args.csv) as f:
        rows = list(csv.DictReader(f))
    lines = ["# per-kernel time, rocprofv3 --kernel-trace --stats",
             "# command: %s" % args.command,
             "%-62s %6s %12s %12s %7s" % ("kernel", "calls", "avg_us", "total_ms", "pct")]
    for r in rows[: args.top]:
        lines.append("%-62s %6s %12.1f %12.2f %7.2f" % (
            r["Name"][:62], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, end="")


def trace(args):
    """Per-kernel time from a --kernel-trace CSV over the steady state: after
    every idle gap of the GPU longer than `gap_ms` (host work between timed
    regions, during which the clocks drop) the first `skip` dispatches of
    each kernel are left out."""
    disp = []
    with open(args.csv) as f:
        for r in csv.DictReader(f):
            disp.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    disp.sort()
    per = collections.defaultdict(list)
    calls = collections.Counter()
    since_gap = collections.Counter()
    last_end = None
    for st, en, name in disp:
        if last_end is not None and st - last_end > args.gap_ms * 1e6:
            since_gap.clear()
        last_end = en if last_end is None else max(last_end, en)
        calls[name] += 1
        since_gap[name] += 1
        if since_gap[name] > args.skip:
            per[name].append((en - st) / 1e3)
    rows = []
    for name in calls:
        durs = per.get(name) or []
        if durs:
            rows.append((sum(durs), name, calls[name], len(durs), durs))
    rows.sort(reverse=True)
    lines = ["# per-kernel time, steady state: after every idle gap over %g ms the first "
             "%d dispatches of each kernel are left out" % (args.gap_ms, args.skip),
             "# command: %s" % args.command,
             "# summary command: python3 -m paper_1306_4161_amd.profiling %s" % shlex.join(
                 sys.argv[1:]),
             "%-64s %6s %6s %11s %11s %11s %11s" % ("kernel", "calls", "kept", "avg_us",
                                                      "min_us", "max_us", "total_ms")]
    for total, name, calls, kept, durs in rows[: args.top]:
        lines.append("%-64s %6d %6d %11.1f %11.1f %11.1f %11.3f" % (
            name[:64], calls, kept, total / kept, min(durs), max(durs), total / 1e3))
    text = "\n".join(lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, end="")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("launches")
    a.add_argument("--path", default="fp64", choices=["fp64", "bf16", "int8"])
    a.add_argument("--n", type=int, default=16384)
    a.add_argument("--P", type=int, default=16)
    a.add_argument("--Q", type=int, default=16)
    a.add_argument("--G", type=int, default=16)
    a.add_argument("--b", type=int, default=256)
    a.add_argument("--M", type=int, default=1024)
    a.add_argument("--sigma", type=float, default=2.0)
    a.add_argument("--count", type=int, default=3)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--source", required=True, help="comma-separated csrc files")
    t.add_argument("--algorithmic", type=float, default=0.0)
    t.add_argument("--fetch-command", default="")
    t.add_argument("--write-command", default="")
    t.add_argument("--out", default="")
    m = sub.add_parser("mfma")
    m.add_argument("csv")
    m.add_argument("--kernel", required=True)
    m.add_argument("--workload", required=True)
    m.add_argument("--source", required=True, help="comma-separated csrc files")
    m.add_argument("--command", default="")
    m.add_argument("--xcds", type=int, default=8)
    m.add_argument("--simds", type=int, default=1024)
    m.add_argument("--out", default="")
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", default="")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--out", default="")
    tr = sub.add_parser("trace")
    tr.add_argument("csv")
    tr.add_argument("--skip", type=int, default=3)
    tr.add_argument("--gap-ms", type=float, default=20.0)
    tr.add_argument("--command", default="")
    tr.add_argument("--top", type=int, default=12)
    tr.add_argument("--out", default="")
    args = ap.parse_args()
    {"launches": launches, "traffic": traffic, "mfma": mfma, "stats": stats,
     "trace": trace}[args.cmd](args)


if __name__ == "__main__":
    main()
