"""Benchmark: Galerkin near-field assembly of the Laplace single- and
double-layer operators on the 8192-triangle octahedron sphere (cluster tree
by bounding-box bisection with leaf size 64, admissibility
max(diam) <= 2 dist, Sauter-Schwab order 4, Duffy/Gauss order 4, plain FP64).

One step = bem_assemble_nearfield for the SLP and for the DLP over all
inadmissible blocks of the block tree, inputs resident in HBM.  Prints one
JSON line (value = entries/s over the whole step) with a roofline object for
the dominant kernel (the DLP block kernel, VALU-bound FP64) measured live
with HIP events on the launch stream, and the FP64 CPU oracle's throughput
on a bounded sample of the same blocks as cpu_baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Galerkin entries/s + H2 setup time at 1e-6 rel err, learned/mixed vs plain FP64"
FP64_VALU_PEAK = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# algorithmic flops per quadrature point (FMA = 2, rsqrt = 1), and the extra
# flops of a Sauter-Schwab point (region map and difference vector)
FLOPS_PER_POINT = {(0, 0): 11.0, (0, 1): 19.0, (1, 0): 18.0, (1, 1): 30.0}
SS_EXTRA = 35.0
SS_REGIONS = {3: 6, 2: 5, 1: 2}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    return p.parse_args()


def class_counts(tri, rows, cols):
    """Pairs per class (0 disjoint, 1 vertex, 2 edge, 3 identical) over blocks."""
    counts = np.zeros(4, dtype=np.int64)
    for r, c in zip(rows, cols):
        tr, tc = tri[r], tri[c]
        sh = np.zeros((r.size, c.size), dtype=np.int8)
        for a in range(3):
            for b in range(3):
                sh += tr[:, a, None] == tc[None, :, b]
        counts += np.bincount(sh.ravel(), minlength=4)[:4]
    return counts


def launch_flops(counts, kernel, layer, q_reg, q_sing):
    f = FLOPS_PER_POINT[(kernel, layer)]
    flops = counts[0] * (q_reg ** 2) ** 2 * f
    for cls, nreg in SS_REGIONS.items():
        flops += counts[cls] * nreg * q_sing ** 4 * (f + SS_EXTRA)
    return float(flops)


def cpu_baseline(m, rows, cols, q, seconds):
    import oracle
    from bem_inputs import sample_subset
    order = sample_subset(np.arange(len(rows)), len(rows), seed=1)
    rng = np.random.Generator(np.random.PCG64(1))
    order = order[rng.permutation(order.size)]
    n = 0
    t0 = time.perf_counter()
    used = 0
    for k in order:
        for layer in (0, 1):
            g = oracle.block(m.v, m.tri, rows[k], cols[k], layer=layer, q_reg=q, q_sing=q)
            n += g.size
        used += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "entries/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{used} of {len(rows)} near blocks (seeded order), SLP and DLP, "
                      f"{n} entries in {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the assembly shards "
              "by blocks with no communication, see the sharding notes; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1510_07244_amd as pk
    from bem_inputs import octahedron_sphere

    q = 4
    m = octahedron_sphere(32)
    ct = pk.ClusterTree(m.v, m.tri, leaf=64)
    near, far = pk.block_tree(ct, eta=2.0)
    rows = [ct.idx(t) for t, s in near]
    cols = [ct.idx(s) for t, s in near]
    counts = class_counts(m.tri, rows, cols)
    ctx = pk.Context(0)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists(rows, cols)
    ops = [pk.make_op(pk.LAPLACE, layer, q_regular=q, q_singular=q) for layer in (pk.SLP, pk.DLP)]
    outs = [torch.empty(total, dtype=torch.float64, device="cuda") for _ in ops]
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]

    def step(events=None):
        for k, (op, out) in enumerate(zip(ops, outs)):
            if events:
                events[2 * k].record(stream)
            ctx.assemble_nearfield(mesh, op, blocks, out, stream=stream)
            if events:
                events[2 * k + 1].record(stream)

    for _ in range(args.warmup):
        step()
    ctx.check(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check(stream)
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_slp = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    ms_dlp = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
    entries = 2 * total
    f_slp = launch_flops(counts, 0, 0, q, q)
    f_dlp = launch_flops(counts, 0, 1, q, q)
    result = {
        "metric": METRIC,
        "value": entries / (ms_step * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "Laplace SLP+DLP near field, octahedron sphere 8192 triangles, leaf 64, "
                        "eta 2, Sauter-Schwab q=4, Duffy/Gauss q=4, plain FP64",
            "triangles": int(m.nt), "near_blocks": int(len(near)), "far_blocks": int(len(far)),
            "entries_per_step": int(entries),
            "pairs_by_class": {"disjoint": int(counts[0]), "vertex": int(counts[1]),
                               "edge": int(counts[2]), "identical": int(counts[3])},
        },
        "roofline": {
            "kernel": "k_blocks<Laplace, DLP> (+ geometry kernel in the same call)",
            "bound": "alu", "achieved": f_dlp / (ms_dlp * 1e-3) / 1e12,
            "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": f_dlp / (ms_dlp * 1e-3) / FP64_VALU_PEAK, "traffic": None,
            "ms_per_launch": ms_dlp, "flops_per_launch": f_dlp,
        },
        "roofline_slp": {
            "kernel": "k_blocks<Laplace, SLP>", "bound": "alu",
            "achieved": f_slp / (ms_slp * 1e-3) / 1e12, "peak": FP64_VALU_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": f_slp / (ms_slp * 1e-3) / FP64_VALU_PEAK,
            "ms_per_launch": ms_slp, "flops_per_launch": f_slp,
        },
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(m, rows, cols, q, args.cpu_seconds)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
