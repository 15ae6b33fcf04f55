"""Tables of the committed rocprofv3 summaries (profiles/*.md) from the raw
rocprofv3 CSV output of bench.py runs.

    python bench_profile.py trace  --csv DIR/..._kernel_trace.csv --bench-log LOG \
        --cmd "COMMAND" --title "TITLE" [--kernel NAME --grid N --flops F] > profiles/X.md
    python bench_profile.py counters --csv DIR/..._counter_collection.csv [...] > ...

trace: per-dispatch durations (End - Start) grouped by kernel name and grid
size (workgroups), in dispatch order, with the mean over all dispatches and
over the last five; with --kernel/--grid/--flops, the roofline of that
launch from the profiler's durations beside the HIP-event duration the same
bench run printed (roofline.ms_per_launch in its JSON line).

counters: per-dispatch counter values of the listed launches (kernel name
and grid size), and the FLOP count the VALU instruction counters give:
64 lanes x (2 FMA + ADD + MUL + TRANS) per wave instruction, per precision.
"""
import argparse
import collections
import csv
import json
import re
import sys


def _kname(raw):
    """Short kernel name: the function and its template arguments."""
    m = re.search(r"(k_\w+)(<[^()]*>)?", raw)
    if not m:
        return raw[:60]
    name = m.group(1) + (m.group(2) or "")
    return re.sub(r"\(\w+\)", "", name).replace("  ", " ")


def _grid_wg(row):
    g = int(row.get("Grid_Size_X") or row.get("Grid_Size") or 0)
    w = int(row.get("Workgroup_Size_X") or row.get("Workgroup_Size") or 1)
    return max(1, g // max(1, w))


def read_trace(path):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    groups = collections.OrderedDict()
    for r in rows:
        key = (_kname(r["Kernel_Name"]), _grid_wg(r))
        groups.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return groups


def bench_json(path):
    """The last JSON line of a bench.py log (None if there is none)."""
    line = None
    for ln in open(path):
        ln = ln.strip()
        if ln.startswith("{") and ln.endswith("}"):
            line = ln
    return json.loads(line) if line else None


def cmd_trace(a):
    groups = read_trace(a.csv)
    out = [f"# {a.title}", "", "Command (repository root, MI355X, one GPU):", "",
           "    export TMPDIR=/tmp", f"    {a.cmd}", "",
           "Per-dispatch durations (End - Start of the kernel trace), grouped by kernel and",
           "grid size in workgroups, in dispatch order; the last five dispatches of a row",
           "are the timed steps when the command times at least five.  Table made by",
           "`bench_profile.py trace` from the run's kernel-trace CSV.", "",
           "| Kernel | Workgroups | Dispatches | Average ns | Average of the last 5 ns | Min ns | Max ns |",
           "|---|---|---|---|---|---|---|"]
    items = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    for (name, wg), d in items[:a.rows]:
        out.append(f"| `{name}` | {wg} | {len(d)} | {sum(d) / len(d):,.0f} | "
                   f"{sum(d[-5:]) / len(d[-5:]):,.0f} | {min(d):,} | {max(d):,} |")
    if a.kernel:
        d = groups.get((a.kernel, a.grid))
        if d is None:
            sys.exit(f"no dispatches of {a.kernel} with {a.grid} workgroups")
        last = d[-5:]
        prof_ms = sum(last) / len(last) / 1e6
        out += ["", f"Roofline of `{a.kernel}` ({a.grid} workgroups), {a.flops:.6g} algorithmic "
                    f"flops per launch, against {a.peak} TFLOP/s:", ""]
        out.append(f"    profiler, mean of the last {len(last)} dispatches: {prof_ms:.4f} ms "
                   f"-> {a.flops / prof_ms / 1e9:.2f} TFLOP/s, frac {a.flops / prof_ms / 1e9 / a.peak:.4f}")
        out.append(f"    profiler, fastest dispatch: {min(d) / 1e6:.4f} ms -> "
                   f"frac {a.flops / (min(d) / 1e6) / 1e9 / a.peak:.4f}")
        if a.bench_log:
            js = bench_json(a.bench_log)
            rl = js.get(a.roofline_key) if js else None
            if rl:
                ev = rl["ms_per_launch"]
                out.append(f"    HIP events in the same run (bench.py {a.roofline_key}): {ev:.4f} ms "
                           f"-> frac {a.flops / ev / 1e9 / a.peak:.4f}")
    print("\n".join(out))


def cmd_counters(a):
    rows = list(csv.DictReader(open(a.csv)))
    per = collections.OrderedDict()
    for r in rows:
        key = (int(r.get("Dispatch_Id", 0)), _kname(r["Kernel_Name"]), _grid_wg(r))
        per.setdefault(key, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    names = sorted({c for v in per.values() for c in v})
    out = [f"# {a.title}", "", "Command (repository root, MI355X, one GPU):", "",
           "    export TMPDIR=/tmp", f"    {a.cmd}", "",
           "Counter values per dispatch (summed over the shader engines), made by",
           "`bench_profile.py counters` from the run's counter-collection CSV.", "",
           "| Dispatch | Kernel | Workgroups | " + " | ".join(names) + " | FP64 FLOP | FP32 FLOP |",
           "|---|---|---|" + "---|" * (len(names) + 2)]
    for (did, name, wg), v in per.items():
        if a.min_grid and wg < a.min_grid:
            continue

        def flop(p):
            return 64 * (2 * v.get(f"SQ_INSTS_VALU_FMA_{p}", 0) + v.get(f"SQ_INSTS_VALU_ADD_{p}", 0) +
                         v.get(f"SQ_INSTS_VALU_MUL_{p}", 0) + v.get(f"SQ_INSTS_VALU_TRANS_{p}", 0))
        out.append(f"| {did} | `{name}` | {wg} | " + " | ".join(f"{v.get(n, 0):.4g}" for n in names) +
                   f" | {flop('F64'):.4g} | {flop('F32'):.4g} |")
    print("\n".join(out))


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--csv", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--rows", type=int, default=40)
    t.add_argument("--kernel")
    t.add_argument("--grid", type=int)
    t.add_argument("--flops", type=float)
    t.add_argument("--peak", type=float, default=78.6)
    t.add_argument("--bench-log")
    t.add_argument("--roofline-key", default="roofline")
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--min-grid", type=int, default=0)
    a = p.parse_args()
    cmd_trace(a) if a.what == "trace" else cmd_counters(a)


if __name__ == "__main__":
    main()
