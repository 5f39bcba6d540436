"""Summaries of rocprofv3 CSV output for the kernels of the convolution sweeps.

    python -m paper_1612_08395_amd.profile_summary trace --dir D --command CMD --out F.md
    python -m paper_1612_08395_amd.profile_summary pmc --fetch D1 --write D2 [--sq D3]
        --command CMD --out F.md [--traffic-json F.json]

`trace` reads `*_kernel_stats.csv` / `*_kernel_trace.csv` of a
`rocprofv3 --kernel-trace --stats --output-format csv` run; `pmc` reads the
`*_counter_collection.csv` of `--pmc FETCH_SIZE`, `--pmc WRITE_SIZE` (and an
optional SQ counter pass) runs.  HBM bytes are calibrated against the plain
device-to-device copy the profiled program makes (`__amd_rocclr_copyBuffer`
of a known size): each counter is scaled by (bytes the copy moves) / (what
the counter reads for it).
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
# sources whose change invalidates stored counter readings of the sweep kernels
SWEEP_SOURCES = ("conv_kernels.h", "fft_lds.h", "wave_fft.h", "col_wave.h", "row_wave.h", "common.h",
                 "launch.h", "conv.hip")
COLUMN_KERNEL = "k_col_conv_w<2048, 2>"
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def kernel_source_sha():
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name, width=72):
    n = re.sub(r"^void ", "", name)
    n = re.sub(r"\(.*", "", n)
    return n if len(n) <= width else n[:width - 3] + "..."


def _one(pattern):
    got = sorted(glob.glob(pattern))
    if not got:
        raise SystemExit(f"no file matches {pattern}")
    return got[0]


def trace(args):
    stats = list(csv.DictReader(open(_one(os.path.join(args.dir, "*kernel_stats.csv")))))
    rows = list(csv.DictReader(open(_one(os.path.join(args.dir, "*kernel_trace.csv")))))
    durs = collections.defaultdict(list)
    for r in rows:
        durs[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = [f"# rocprofv3 kernel trace: {args.title}", "",
           "Command:", "", "```", args.command, "```", "",
           f"Dispatches: {len(rows)}", "",
           "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for s in sorted(stats, key=lambda s: -float(s["TotalDurationNs"]))[:args.top]:
        out.append(f"| `{short(s['Name'])}` | {s['Calls']} | {float(s['AverageNs']) / 1e3:.2f} | "
                   f"{float(s['TotalDurationNs']) / 1e6:.2f} | {float(s['Percentage']):.1f} |")
    out += ["", "Launches that did work vs launches that returned at once (a solver chunk "
            "queued past convergence; every kernel of the loop first reads the stop flag). "
            "Split at half the median duration of the kernel:", "",
            "| kernel | working | avg us (working) | early exits | avg us (early) |",
            "|---|---:|---:|---:|---:|"]
    focus = {}
    for name, d in sorted(durs.items(), key=lambda x: -sum(x[1]))[:args.top]:
        med = statistics.median(d)
        work = [x for x in d if x >= 0.5 * med]
        early = [x for x in d if x < 0.5 * med]
        out.append(f"| `{short(name)}` | {len(work)} | {statistics.fmean(work):.2f} | {len(early)} | "
                   f"{statistics.fmean(early) if early else 0.0:.2f} |")
        if args.focus and args.focus in name:
            focus = {"kernel": short(name, 200), "working_launches": len(work),
                     "avg_us_working": statistics.fmean(work), "early_exits": len(early),
                     "avg_us_all": statistics.fmean(d)}
    if focus:
        out += ["", f"Focus kernel `{focus['kernel']}`: {focus['working_launches']} working "
                f"launches, mean {focus['avg_us_working']:.2f} us "
                f"(all {focus['working_launches'] + focus['early_exits']} launches: "
                f"{focus['avg_us_all']:.2f} us)."]
    if args.bench_json and focus:
        with open(args.bench_json) as fh:
            b = json.loads([ln for ln in fh if ln.startswith("{")][-1])
        r = b["roofline"]
        out += ["", f"The same run's bench.py line (HIP events on the solver stream around "
                f"each column launch of one sweep of the timed workload): "
                f"{r['ms_per_launch'] * 1e3:.2f} us per "
                f"launch over {r['launches_timed']} launches, {r['achieved']} GB/s algorithmic "
                f"({r['frac']} of {r['peak']} GB/s); trace mean of working launches "
                f"{focus['avg_us_working']:.2f} us.  The event figure includes the dispatch gap "
                f"between back-to-back launches; solves/s of this traced run: {b['value']}."]
    if args.note:
        out += ["", args.note]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def _counters(d):
    """Per kernel and counter: the values of the dispatches that did work.  A
    dispatch whose duration is under half the median of its kernel is a
    launch queued past the solver's convergence that returned at once (every
    CG kernel first reads the stop flag); those are counted, not averaged."""
    rows = list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))
    per = collections.defaultdict(list)
    grid = {}
    for r in rows:
        key = r["Kernel_Name"]
        dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        per[(key, r["Counter_Name"])].append((dur, float(r["Counter_Value"])))
        grid[key] = int(r["Grid_Size"])
    acc = collections.defaultdict(dict)
    early = collections.defaultdict(int)
    for (key, cname), recs in per.items():
        med = statistics.median(x[0] for x in recs)
        acc[key][cname] = [v for t, v in recs if t >= 0.5 * med]
        early[key] = len(recs) - len(acc[key][cname])
    return acc, grid, early


def pmc(args):
    fetch, grid, early = _counters(args.fetch)
    write, _, _ = _counters(args.write)
    copy_bytes = args.copy_bytes
    cf = [v for k, c in fetch.items() if k.startswith(COPY_KERNEL) for v in c["FETCH_SIZE"]]
    cw = [v for k, c in write.items() if k.startswith(COPY_KERNEL) for v in c["WRITE_SIZE"]]
    big_f = max(cf)
    big_w = max(cw)
    sf = copy_bytes / (big_f * 1024.0)
    sw = copy_bytes / (big_w * 1024.0)
    out = [f"# rocprofv3 HBM counters: {args.title}", "", "Commands:", "", "```", args.command,
           "```", "",
           f"Calibration: a device copy of {copy_bytes} bytes each way reads FETCH_SIZE = "
           f"{big_f:.1f} KiB and WRITE_SIZE = {big_w:.1f} KiB, so bytes = FETCH_SIZE x 1024 x "
           f"{sf:.3f} and WRITE_SIZE x 1024 x {sw:.3f}.", "",
           "Means over the dispatches that did work; 'early' counts launches queued past "
           "the solver's convergence (duration under half the kernel's median), which read "
           "and write next to nothing.", "",
           "| kernel | grid | launches | early | FETCH KiB | WRITE KiB | calibrated MB/launch |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    traffic = {}
    for k in sorted(fetch, key=lambda k: -statistics.fmean(fetch[k]["FETCH_SIZE"])):
        if k not in write or k.startswith(COPY_KERNEL):
            continue
        f = statistics.fmean(fetch[k]["FETCH_SIZE"])
        w = statistics.fmean(write[k]["WRITE_SIZE"])
        mb = (f * 1024 * sf + w * 1024 * sw) / 1e6
        if mb < 0.01:
            continue
        out.append(f"| `{short(k)}` | {grid[k]} | {len(fetch[k]['FETCH_SIZE'])} | {early[k]} | "
                   f"{f:.1f} | {w:.1f} | {mb:.2f} |")
        if COLUMN_KERNEL in k:
            traffic = {"kernel": short(k, 200), "bytes_per_launch": round(mb * 1e6),
                       "fetch_bytes": round(f * 1024 * sf), "write_bytes": round(w * 1024 * sw),
                       "fetch_scale": sf, "write_scale": sw, "source_sha": kernel_source_sha(),
                       "command": args.command}
    if args.sq:
        sq, _, _ = _counters(args.sq)
        names = sorted({c for k in sq for c in sq[k]})
        out += ["", "SQ counters (mean per launch):", "",
                "| kernel | " + " | ".join(names) + " |", "|---|" + "---:|" * len(names)]
        for k in sorted(sq):
            if k.startswith("__amd") or "FillFunctor" in k:
                continue
            out.append(f"| `{short(k)}` | " +
                       " | ".join(f"{statistics.fmean(sq[k][c]):.4g}" for c in names) + " |")
    if args.note:
        out += ["", args.note]
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))
    if args.traffic_json and traffic:
        with open(args.traffic_json, "w") as fh:
            json.dump(traffic, fh, indent=1)
            fh.write("\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--focus", default=COLUMN_KERNEL)
    t.add_argument("--bench-json", help="stdout of the traced bench.py run")
    p = sub.add_parser("pmc")
    p.add_argument("--fetch", required=True)
    p.add_argument("--write", required=True)
    p.add_argument("--sq")
    p.add_argument("--copy-bytes", type=int, default=4 << 28)
    p.add_argument("--traffic-json")
    for s in (t, p):
        s.add_argument("--command", required=True)
        s.add_argument("--out", required=True)
        s.add_argument("--title", default="")
        s.add_argument("--top", type=int, default=20)
        s.add_argument("--note", default="")
    args = ap.parse_args()
    (trace if args.mode == "trace" else pmc)(args)


if __name__ == "__main__":
    main()
