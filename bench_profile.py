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

traffic: the block-kernel launches of `bench.py --counter-pass` (near field
of each layer, the double layer's coupling, the one-pass near field) from
its counter passes -- HBM bytes from FETCH_SIZE and WRITE_SIZE, each scaled
by its reading of the pass's closing 512 MiB copy, counted FLOPs, issue
counters -- beside the algorithmic bytes and flops and the durations of the
same launches in a kernel trace of the bench; ends with the values bench.py
reads for roofline.traffic and the hash of the sources they stay valid for.
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


def _counter_rows(path):
    """(kernel, workgroups) -> list of {counter: value} per dispatch, in
    dispatch order (with the dispatch's duration under the counters, ns, as
    'duration_ns')."""
    per = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        key = (int(r["Dispatch_Id"]), _kname(r["Kernel_Name"]), _grid_wg(r))
        d = per.setdefault(key, {})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            d["duration_ns"] = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = collections.OrderedDict()
    for (_, name, wg), v in sorted(per.items()):
        out.setdefault((name, wg), []).append(v)
    return out


def cmd_traffic(a):
    import hashlib
    import os
    runs = [_counter_rows(p) for p in a.csv]
    trace = read_trace(a.trace) if a.trace else {}
    js = bench_json(a.bench_log) if a.bench_log else None
    # the launches, identified by kernel and workgroups (k-th occurrence)
    launches = [("SLP near field (2400 blocks)", "k_blocks<0, 0, 8, false>", 2400, 0,
                 a.near_entries * 8, None),
                ("DLP near field (2400 blocks)", "k_blocks<0, 1, 8, false>", 2400, 0,
                 a.near_entries * 8, "near_per_layer.roofline_dlp"),
                ("DLP coupling (3760 blocks)", "k_blocks<0, 1, 8, false>", 3760, 0,
                 a.coupling_entries * 8, "roofline"),
                ("SLP+DLP near field, one pass (1292 blocks)", "k_blocks<0, 2, 8, false>", 1292, 0,
                 2 * a.near_entries * 8, "roofline_near_both"),
                ("SLP coupling, mirrored (1880 blocks)", "k_blocks<0, 0, 8, false>", 1880, 0,
                 2 * a.slp_coupling_entries * 8, "roofline_slp_coupling"),
                ("Helmholtz kappa 4 DLP coupling, q 5 (3760 blocks)", "k_blocks<1, 1, 5, false>",
                 3760, 0, a.helmholtz_dlp_entries * 16, None),
                ("Helmholtz kappa 4 SLP coupling, q 5, mirrored (1880 blocks)",
                 "k_blocks<1, 0, 5, false>", 1880, 0, 2 * a.helmholtz_slp_entries * 16, None)]

    def value(name, wg, k, counter):
        for run in runs:
            v = run.get((name, wg))
            if v and k < len(v) and counter in v[k]:
                return v[k][counter]
        return None

    # calibration: the largest copy of the pass (512 MiB read and written)
    copies = [v for run in runs for (n, wg), vs in run.items() if n == "__amd_rocclr_copyBuffer"
              for v in vs]
    cf = max((c["FETCH_SIZE"] for c in copies if "FETCH_SIZE" in c), default=None)
    cw = max((c["WRITE_SIZE"] for c in copies if "WRITE_SIZE" in c), default=None)
    kib = a.copy_bytes / 1024
    fs, ws = kib / cf, kib / cw
    out = [f"# {a.title}", "", "Commands (repository root, MI355X, one GPU; one counter pass per run):",
           "", "    export TMPDIR=/tmp"] + [f"    {c}" for c in a.cmd] + ["",
           "Made by `bench_profile.py traffic` from the runs' counter-collection CSVs (and the",
           "kernel trace and JSON line of a bench run for durations and algorithmic flops).", "",
           f"Calibration: the pass's closing copy of {a.copy_bytes} bytes reads FETCH_SIZE = "
           f"{cf:.0f} KiB and WRITE_SIZE = {cw:.0f} KiB, so FETCH_SIZE is scaled by {fs:.4f} and "
           f"WRITE_SIZE by {ws:.4f}.", "",
           "| Launch | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) | algorithmic bytes "
           "(output) | write / output | SQ_INSTS_VALU | SQ_INSTS_LDS | FP64 FLOP counted | "
           "FP32 FLOP counted | algorithmic FLOP | counted / algorithmic | ms (trace, last 5; "
           "else the FLOP pass) | "
           "counted TFLOP/s | counted / measured FP64 peak |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    peak = None  # TFLOP/s, bem_valu_peak in the bench run of the trace
    if js and isinstance(js.get("roofline"), dict):
        peak = js["roofline"].get("peak_measured")
    stored = None
    for label, name, wg, k, out_bytes, key in launches:
        f, w = value(name, wg, k, "FETCH_SIZE"), value(name, wg, k, "WRITE_SIZE")
        hbm = 1024 * (f * fs + w * ws) if f is not None and w is not None else None

        def flop(p):
            parts = [value(name, wg, k, f"SQ_INSTS_VALU_{x}_{p}") for x in ("FMA", "ADD", "MUL",
                                                                        "TRANS")]
            if any(x is None for x in parts):
                return None
            return 64 * (2 * parts[0] + parts[1] + parts[2] + parts[3])
        f64, f32 = flop("F64"), flop("F32")
        model = None
        if js and key:
            node = js
            for part in key.split("."):
                node = node.get(part) if isinstance(node, dict) else None
            model = node.get("flops_per_launch") if isinstance(node, dict) else None
        d = trace.get((name, wg))
        ms = sum(d[-5:]) / len(d[-5:]) / 1e6 if d else None
        if ms is None:  # not in the trace: the FLOP pass's own duration
            for run in runs:
                v = run.get((name, wg))
                if v and k < len(v) and "SQ_INSTS_VALU_FMA_F64" in v[k] and "duration_ns" in v[k]:
                    ms = v[k]["duration_ns"] / 1e6
        fmt = lambda x, spec: "-" if x is None else format(x, spec)
        out.append(f"| {label} | {fmt(f, '.0f')} | {fmt(w, '.0f')} | {fmt(hbm, '.4g')} | "
                   f"{out_bytes:.4g} | {fmt(None if w is None else 1024 * w * ws / out_bytes, '.2f')} | "
                   f"{fmt(value(name, wg, k, 'SQ_INSTS_VALU'), '.4g')} | "
                   f"{fmt(value(name, wg, k, 'SQ_INSTS_LDS'), '.4g')} | {fmt(f64, '.4g')} | "
                   f"{fmt(f32, '.4g')} | {fmt(model, '.4g')} | "
                   f"{fmt(None if model is None or f64 is None else (f64 + (f32 or 0)) / model, '.3f')} | "
                   f"{fmt(ms, '.4f')} | {fmt(None if ms is None or f64 is None else f64 / ms / 1e9, '.2f')} | "
                   f"{fmt(None if ms is None or f64 is None or not peak else f64 / ms / 1e9 / peak, '.2f')} |")
        if key == "roofline":
            stored = (f, w, f64)
    out += ["", f"Algorithmic output: near field {a.near_entries:,} FP64 entries = "
                f"{a.near_entries * 8 / 1e6:.1f} MB per launch and layer; DLP coupling "
                f"{a.coupling_entries:,} entries = {a.coupling_entries * 8 / 1e6:.1f} MB.",
            "Counted FLOP = 64 lanes x (2 FMA + ADD + MUL + TRANS) per wave instruction; the",
            "algorithmic FLOP are bench.py's model (the roofline numerator): counted over model",
            "is the instruction overhead of the reciprocal square root, its Newton step and the",
            "quadrature bookkeeping.  The measured FP64 peak is bem_valu_peak's in the bench run",
            f"of the trace ({peak:.1f} TFLOP/s): the headline fraction of counted FLOP." if peak else
            "No measured peak in the bench log.", ""]
    h = hashlib.sha256()
    for src in a.sources:
        h.update(open(os.path.join(a.root, src), "rb").read())
    out += ["Values read by bench.py (roofline.traffic of the DLP coupling launch, bytes",
            "per launch; valid while the sources below hash to this value):", "",
            f"    source_sha256: {h.hexdigest()}", f"    sources: {' '.join(a.sources)}",
            f"    fetch_kib_per_launch: {stored[0]:.0f}", f"    write_kib_per_launch: {stored[1]:.0f}",
            f"    fetch_scale: {fs:.6f}", f"    write_scale: {ws:.6f}",
            f"    fp64_flop_counted_per_launch: {stored[2]:.6g}"]
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
    r = sub.add_parser("traffic")
    r.add_argument("--csv", nargs="+", required=True, help="counter-collection CSVs")
    r.add_argument("--cmd", nargs="+", required=True)
    r.add_argument("--title", required=True)
    r.add_argument("--trace")
    r.add_argument("--bench-log")
    r.add_argument("--near-entries", type=int, required=True)
    r.add_argument("--coupling-entries", type=int, required=True)
    r.add_argument("--slp-coupling-entries", type=int, default=0,
                   help="evaluated entries of the mirrored single-layer coupling launch")
    r.add_argument("--helmholtz-dlp-entries", type=int, default=0)
    r.add_argument("--helmholtz-slp-entries", type=int, default=0,
                   help="evaluated entries of the mirrored Helmholtz single-layer coupling")
    r.add_argument("--copy-bytes", type=int, default=512 * 1024 * 1024)
    r.add_argument("--sources", nargs="+", required=True)
    r.add_argument("--root", default=".")
    a = p.parse_args()
    {"trace": cmd_trace, "counters": cmd_counters, "traffic": cmd_traffic}[a.what](a)


if __name__ == "__main__":
    main()
