"""Benchmark: H^2-matrix setup of the Laplace single- and double-layer
operators on the 8192-triangle octahedron sphere (cluster tree by bounding-box
bisection, leaf size 64; admissibility max(diam) <= 2 dist; Sauter-Schwab and
Duffy/Gauss order 4; Green quadrature order 4 on each face of the Green box;
cross-approximation tolerance 5e-8, which keeps sampled admissible blocks
within 1e-6 relative error of the dense FP64 oracle -- checked by the GPU
tests; plain FP64).

Setup (timed once per repeat, wall clock, host pivot search included):
cluster/block trees, nested row basis (Green matrices side 0) and the
double layer's column basis (side 1), each level: Green matrices on the GPU,
cross approximation on the host, basis contraction on the matrix cores; then
near-field and coupling blocks of both operators.

One step (the data-parallel hot path, inputs resident in HBM, pivots as
chosen by the setup): Green matrices and basis contractions of both bases,
near-field blocks of SLP and DLP (one pass for both layers over the blocks
with t <= s), coupling blocks of SLP and DLP (the single layer's blocks of a
pair (t, s), (s, t), t != s, evaluated once, the other written as the
transpose).  The four phases are independent (the pivots are fixed): the
timed step runs them on four streams; phase_ms comes from the same step on
one stream.  value = Galerkin entries written (near field + coupling) per
second; entries_evaluated_per_step counts those evaluated.  The roofline object is
for the dominant kernel, the double layer's coupling launch (VALU-bound
FP64, the step's longest), measured with HIP events on its launch stream; cpu_baseline is the FP64 CPU
oracle on a bounded sample of the same blocks.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--one-stream]
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Galerkin entries/s + H2 setup time at 1e-6 rel err, learned/mixed vs plain FP64"
FP64_VALU_PEAK = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# Algorithmic flops (FMA = 2, rsqrt = sincos = 1) per regular point pair,
# by (kernel, layer); a Sauter-Schwab point of the factored rule adds the
# difference vector d(eta) = 4 scaled edge vectors (24 flops).
FLOPS_PER_POINT = {(0, 0): 11.0, (0, 1): 19.0, (1, 0): 18.0, (1, 1): 30.0}
SS_EXTRA = 24.0
SS_REGIONS = {3: 6, 2: 5, 1: 2}
Q = 4
FP32_VALU_PEAK = 157.3e12  # published, with packed FP32 (the library is compiled without it)
MIXED_RATIO = 0.5  # mixed form: pairs with box gap < 0.5 max diameter stay FP64


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_blocks_sphere8192.md")


def stored_counters():
    """(HBM bytes, counted FP64 flops) per DLP coupling launch from the
    committed counter passes (FETCH_SIZE and WRITE_SIZE, each scaled by its
    reading of a copy of known size; the SQ_INSTS_VALU_*_F64 counters), or
    (None, None) if the block kernel's sources changed since."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and line.startswith("    "):
                k, v = line.strip().split(":", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in kv["sources"].split():
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != kv["source_sha256"]:
            return None, None
        traffic = 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_scale"]) +
                            float(kv["write_kib_per_launch"]) * float(kv["write_scale"]))
        flops = float(kv["fp64_flop_counted_per_launch"]) if "fp64_flop_counted_per_launch" in kv \
            else None
        return traffic, flops
    except (OSError, KeyError, ValueError):
        return None, None


def stored_traffic():
    return stored_counters()[0]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=30)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--setup-repeats", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-helmholtz", action="store_true",
                   help="skip the Helmholtz near-field leg (32768-triangle sphere)")
    p.add_argument("--one-stream", action="store_true",
                   help="time the step on one stream only (for kernel traces, where "
                        "overlapping launches would stretch each other's durations)")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--batched-meshes", type=int, default=64)
    p.add_argument("--learned-group", type=int, default=4,
                   help="rows of a column per network evaluation in the learned legs")
    p.add_argument("--learned-n", type=int, default=128,
                   help="octahedron subdivision of the learned-form sphere (nt = 8 n^2)")
    p.add_argument("--counter-pass", action="store_true",
                   help="for hardware-counter runs: the block launches of the 8192-triangle "
                        "sphere's Laplace step (and the Helmholtz kappa 4 coupling launches), "
                        "then a 512 MiB device copy that calibrates FETCH_SIZE / WRITE_SIZE; "
                        "prints no JSON")
    return p.parse_args()


def counter_pass(torch, pk, ctx, m):
    """The launches the committed traffic counters are read from: the
    per-layer near-field calls with the full lists (SLP, then DLP), the
    double layer's coupling launch of the H2 setup, the one-pass near field of
    both layers on the mirrored list (as the step makes it), then a copy of
    known size."""
    from paper_1510_07244_amd.h2 import H2Setup
    ct = pk.ClusterTree(m.v, m.tri, leaf=64)
    near, _ = pk.block_tree(ct, eta=2.0)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    blocks, total = pk.Blocks.from_lists([ct.idx(t) for t, s in near],
                                         [ct.idx(s) for t, s in near])
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    for layer in (pk.SLP, pk.DLP):
        ctx.assemble_nearfield(mesh, pk.make_op(pk.LAPLACE, layer, q_regular=Q, q_singular=Q),
                               blocks, out)
    ctx.check()
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=Q, q_singular=Q)
    V, W = h.bases((0, 1))
    cd, n_cd = h.coupling_blocks(V, W)
    cout = torch.empty(n_cd, dtype=torch.float64, device="cuda")
    ctx.assemble_coupling(h.mesh, h.op(pk.DLP), cd, cout)
    half, tot = h.near_blocks(mirror=True)
    o1 = torch.empty(tot, dtype=torch.float64, device="cuda")
    o2 = torch.empty_like(o1)
    ctx.assemble_nearfield_both(h.mesh, h.op(pk.SLP), half, o1, o2)
    # the single layer's mirrored coupling launch (the step's), then the
    # Helmholtz coupling launches of config 3's kernel on this mesh
    cs, n_cs = h.coupling_blocks(V, V, mirror=True)
    ctx.assemble_coupling(h.mesh, h.op(pk.SLP), cs, torch.empty(n_cs, dtype=torch.float64,
                                                                 device="cuda"))
    hh = H2Setup(ctx, m.v, m.tri, kernel=pk.HELMHOLTZ, kappa=4.0, q_regular=5, q_singular=5)
    Vh, Wh = hh.bases((0, 1))
    cdh, n_cdh = hh.coupling_blocks(Vh, Wh)
    csh, n_csh = hh.coupling_blocks(Vh, Vh, mirror=True)
    ctx.assemble_coupling(hh.mesh, hh.op(pk.DLP), cdh,
                          torch.empty(n_cdh, dtype=torch.complex128, device="cuda"))
    ctx.assemble_coupling(hh.mesh, hh.op(pk.SLP), csh,
                          torch.empty(n_csh, dtype=torch.complex128, device="cuda"))
    ctx.check()
    a = torch.ones(1 << 26, dtype=torch.float64, device="cuda")  # 512 MiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"near-field entries per launch {total}, DLP coupling entries {n_cd}, "
          f"SLP coupling entries {n_cs // 2} evaluated, Helmholtz DLP / SLP coupling entries "
          f"{n_cdh} / {n_csh // 2}, copy bytes {a.numel() * 8}", flush=True)


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


def mirrored_counts(h, tri):
    """Pair classes of the near field as the mirrored lists evaluate it:
    `eval` the pairs (i, j) evaluated (blocks with t < s, and the entries with
    row >= column of the blocks (t, t)), `trans` their transposed pairs
    (j, i) (those blocks' pairs, the diagonal blocks' with row > column)."""
    ev = np.zeros(4, dtype=np.int64)
    tr_ = np.zeros(4, dtype=np.int64)
    for t, s in h.near:
        if t > s:
            continue
        r, c = h.ct.idx(t), h.ct.idx(s)
        a, b = tri[r], tri[c]
        sh = np.zeros((r.size, c.size), dtype=np.int8)
        for x in range(3):
            for y in range(3):
                sh += a[:, x, None] == b[None, :, y]
        if t < s:
            cnt = np.bincount(sh.ravel(), minlength=4)[:4]
            ev += cnt
            tr_ += cnt
        else:
            ev += np.bincount(sh[np.tril_indices(r.size)], minlength=4)[:4]
            tr_ += np.bincount(sh[np.tril_indices(r.size, -1)], minlength=4)[:4]
    return ev, tr_


def near_flops(counts, kernel, layer, q_reg, q_sing):
    """Laplace: the singular xi sums are moments, q^3 eta points per region.
    Identical pairs: the single layer needs 3 of the 6 regions (the others
    are their mirror images), the double layer none (its entry vanishes on a
    flat triangle)."""
    f = FLOPS_PER_POINT[(kernel, layer)]
    flops = counts[0] * (q_reg ** 2) ** 2 * f
    for cls, nreg in SS_REGIONS.items():
        if cls == 3:
            nreg = 3 if layer == 0 else 0
        pts = nreg * q_sing ** 3 * (1 if kernel == 0 else q_sing)
        flops += counts[cls] * pts * (f + SS_EXTRA)
    return float(flops)


class H2Bench:
    def __init__(self, pk, ctx, m, mixed=False, kernel=0, kappa=0.0, q=Q):
        import torch
        from paper_1510_07244_amd.h2 import H2Setup
        self.pk, self.ctx, self.m = pk, ctx, m
        self.mixed, self.kernel, self.kappa, self.q = mixed, kernel, kappa, q
        sync = torch.cuda.synchronize
        t0 = time.perf_counter()
        self.h = h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=q,
                             q_singular=q)
        t1 = time.perf_counter()
        self.V, self.W = h.bases((0, 1))
        sync()
        t2 = time.perf_counter()
        self.near, self.n_near = h.near_blocks()
        # single layer: of the near-field pairs (t, s), (s, t), t != s, only
        # t < s is evaluated, the other written as its transpose
        self.near_s, _ = h.near_blocks(mirror=True)
        # single layer: of (t, s), (s, t) only t < s is evaluated, the other
        # block is written as its transpose
        self.cs, self.n_cs = h.coupling_blocks(self.V, self.V, mirror=True)
        self.cd, self.n_cd = h.coupling_blocks(self.V, self.W)
        self.ops = [h.op(pk.SLP), h.op(pk.DLP)]
        if mixed:  # regular pairs in FP32, singular and near-singular in FP64
            for op in self.ops:
                op.precision = pk.MIXED
                op.near_singular_ratio = MIXED_RATIO
        dt = dict(dtype=pk.out_dtype(self.ops[0]), device="cuda")
        self.out = {k: torch.empty(n, **dt) for k, n in
                    (("ns", self.n_near), ("nd", self.n_near), ("cs", self.n_cs), ("cd", self.n_cd))}
        # the near field of both layers in one pass over the mirrored list
        self.phases = ["bases", "nb", "cs", "cd"]
        self.assemble()
        ctx.check()
        t3 = time.perf_counter()
        self.t_tree, self.t_bases, self.t_assembly = t1 - t0, t2 - t1, t3 - t2
        self.t_setup = t3 - t0
        # (outside the timed setup) the mirrored single layer evaluates the
        # blocks with t <= s, plus the edge-adjacent entries of the others (as
        # (j, i))
        self.ev_pairs, self.tr_pairs = mirrored_counts(h, m.tri)
        self.near_evaluated_slp = int(self.ev_pairs.sum() + self.tr_pairs[2])

    def near_calls(self, stream=None):
        ctx, h, o = self.ctx, self.h, self.out
        return {
            "nb": lambda: ctx.assemble_nearfield_both(h.mesh, self.ops[0], self.near_s, o["ns"],
                                                      o["nd"], stream),
            "ns": lambda: ctx.assemble_nearfield(h.mesh, self.ops[0], self.near_s, o["ns"], stream),
            "nd": lambda: ctx.assemble_nearfield(h.mesh, self.ops[1], self.near, o["nd"], stream),
        }

    def assemble(self, stream=None, ev=None):
        ctx, h, o = self.ctx, self.h, self.out
        near = self.near_calls(stream)
        seq = [(k, near[k]) for k in self.phases if k in near]
        seq += [("cs", lambda: ctx.assemble_coupling(h.mesh, self.ops[0], self.cs, o["cs"], stream)),
                ("cd", lambda: ctx.assemble_coupling(h.mesh, self.ops[1], self.cd, o["cd"], stream))]
        for name, call in seq:
            if ev:
                ev[name][0].record(stream)
            call()
            if ev:
                ev[name][1].record(stream)

    def step(self, stream, ev=None):
        if ev:
            ev["bases"][0].record(stream)
        self.h.basis_replay(self.V, stream)
        self.h.basis_replay(self.W, stream)
        if ev:
            ev["bases"][1].record(stream)
        self.assemble(stream, ev)

    def step_concurrent(self, torch, main):
        """The same step with its four independent phases (bases, near field,
        single- and double-layer coupling) on four streams, each with a
        context of its own (own geometry scratch and flags), joined on
        `main`: launch tails and the latency-bound basis kernels overlap with
        the other phases."""
        if not hasattr(self, "cctx"):
            self.cctx = [self.ctx] + [self.pk.Context(0) for _ in range(3)]
            self.cstreams = [torch.cuda.Stream() for _ in range(4)]
        h, o = self.h, self.out
        c0, c1, c2, c3 = self.cctx
        s0, s1, s2, s3 = self.cstreams
        start = torch.cuda.Event()
        start.record(main)
        for st in self.cstreams:
            st.wait_event(start)
        c3.assemble_coupling(h.mesh, self.ops[1], self.cd, o["cd"], s3)
        c2.assemble_coupling(h.mesh, self.ops[0], self.cs, o["cs"], s2)
        c1.assemble_nearfield_both(h.mesh, self.ops[0], self.near_s, o["ns"], o["nd"], s1)
        h.basis_replay(self.V, s0)
        h.basis_replay(self.W, s0)
        for st in self.cstreams:
            e = torch.cuda.Event()
            e.record(st)
            main.wait_event(e)

    def check_concurrent(self):
        for c, st in zip(self.cctx, self.cstreams):
            c.check(st)

    def entries(self):
        return 2 * self.n_near + self.n_cs + self.n_cd

    def entries_evaluated(self):
        # the single layer's mirrored blocks are written, not evaluated (apart
        # from the near field's edge-adjacent entries)
        return self.near_evaluated_slp + self.n_near + self.n_cs // 2 + self.n_cd


class BatchedBench:
    """Batched form: near-field and coupling blocks of the Laplace single
    layer on `count` seeded perturbed spheres (512..8192 triangles,
    log-uniform), each with its own H^2 setup, assembled by one persistent
    graph-captured launch (autotuned) against the per-call loop."""

    def __init__(self, pk, ctx, count):
        import torch
        from bem_inputs import perturbed_sphere_batch
        from paper_1510_07244_amd.h2 import H2Setup
        self.pk, self.ctx = pk, ctx
        self.meshes = perturbed_sphere_batch(count)
        t0 = time.perf_counter()
        self.items, self.bases = [], []
        for m in self.meshes:
            h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=Q, q_singular=Q)
            V = h.basis(0)
            self.bases.append(V)
            near, n_near = h.near_blocks(mirror=True)
            cs, n_cs = h.coupling_blocks(V, V, mirror=True)
            self.items.append((h, near, n_near, cs, n_cs))
        torch.cuda.synchronize()
        self.t_bases = time.perf_counter() - t0
        self.op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=Q, q_singular=Q)
        dt = dict(dtype=torch.float64, device="cuda")
        self.out = [(torch.empty(n_near, **dt), torch.empty(n_cs, **dt))
                    for h, near, n_near, cs, n_cs in self.items]
        entries = []
        for (h, near, n_near, cs, n_cs), (on, oc) in zip(self.items, self.out):
            entries += [(h.mesh, near, on, 0), (h.mesh, cs, oc, 1)]
        cache = os.path.join(tempfile.gettempdir(), f"bem_tune_{os.getpid()}.txt")
        t1 = time.perf_counter()
        first = pk.Plan(ctx, self.op, entries, autotune=True, cache=cache)
        torch.cuda.synchronize()
        self.t_plan = time.perf_counter() - t1
        self.tuned = first.config
        first.close()
        # the same plan again with the tuning cached (a later run on this
        # device and operator): lists, queue and graph only
        t1 = time.perf_counter()
        self.plan = pk.Plan(ctx, self.op, entries, autotune=True, cache=cache)
        torch.cuda.synchronize()
        self.t_plan_cached = time.perf_counter() - t1
        os.remove(cache)
        self.n_entries = sum(n_near + n_cs for h, near, n_near, cs, n_cs in self.items)
        self.triangles = sum(m.nt for m in self.meshes)
        # model flops of what one replay evaluates: per mesh the mirrored
        # near field (blocks with t <= s, edge-adjacent transposed pairs
        # evaluated as (j, i)) and half of the mirrored coupling entries
        self.flops = 0.0
        for (h, near, n_near, cs, n_cs), m in zip(self.items, self.meshes):
            ev, tr_ = mirrored_counts(h, m.tri)
            ev = ev.copy()
            ev[2] += tr_[2]
            self.flops += near_flops(ev, 0, 0, Q, Q) + float(n_cs // 2) * Q ** 4 * FLOPS_PER_POINT[(0, 0)]

    def per_call(self, stream):
        for (h, near, n_near, cs, n_cs), (on, oc) in zip(self.items, self.out):
            self.ctx.assemble_nearfield(h.mesh, self.op, near, on, stream)
            self.ctx.assemble_coupling(h.mesh, self.op, cs, oc, stream)

    def batched(self, stream):
        self.plan.run(stream)

    def time(self, torch, fn, stream, steps, warmup):
        for _ in range(warmup):
            fn(stream)
        self.ctx.check(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3 / steps
        self.ctx.check(stream)
        return dt

    def cpu_oracle(self, seconds):
        """The oracle's rate (all host threads) on a seeded sample of the
        meshes' near-field and coupling blocks (single layer)."""
        import oracle
        oracle.use_native_build()
        work = []
        for m, (h, *_), V in zip(self.meshes, self.items, self.bases):
            work += [(m, h.ct.idx(t), h.ct.idx(s)) for t, s in h.near]
            work += [(m, V.piv[t], V.piv[s]) for t, s in h.far]
        order = np.random.Generator(np.random.PCG64(3)).permutation(len(work))
        n = used = 0
        t0 = time.perf_counter()
        for k in order:
            m, r, c = work[k]
            n += oracle.block(m.v, m.tri, r, c, layer=0, q_reg=Q, q_sing=Q).size
            used += 1
            if time.perf_counter() - t0 > seconds:
                break
        dt = time.perf_counter() - t0
        return {"value": n / dt, "unit": "entries/s", "cores": oracle.num_threads(),
                "kind": "oracle", "sample": f"{used} of {len(work)} blocks of the "
                                            f"{len(self.meshes)} meshes (seeded order): {n} "
                                            f"entries in {dt:.1f} s"}

    def result(self, torch, stream, steps, warmup, cpu_seconds=0.0):
        ms_b = self.time(torch, self.batched, stream, steps, warmup)
        ms_p = self.time(torch, self.per_call, stream, steps, warmup)
        sizes = [int(m.nt) for m in self.meshes]
        extra = {"cpu_oracle": self.cpu_oracle(cpu_seconds)} if cpu_seconds > 0 else {}
        return {**extra,
            "value": self.n_entries / (ms_b * 1e-3), "unit": "entries/s", "ms_per_step": ms_b,
            "per_call_ms_per_step": ms_p, "per_call_value": self.n_entries / (ms_p * 1e-3),
            "speedup_vs_per_call": ms_p / ms_b, "entries_per_step": int(self.n_entries),
            "workload": f"Laplace SLP near field + coupling blocks of {len(sizes)} perturbed "
                        f"spheres ({min(sizes)}..{max(sizes)} triangles, {self.triangles} total), "
                        "each with its own H2 setup (leaf 64, eta 2, ACA 5e-8), plain FP64",
            "roofline": {"bound": "alu", "achieved": self.flops / (ms_b * 1e-3) / 1e12,
                         "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                         "frac": self.flops / (ms_b * 1e-3) / FP64_VALU_PEAK,
                         "flops_per_launch": self.flops, "ms_per_launch": ms_b,
                         "kernel": "k_persistent<Laplace, SLP> (one replay: near field and "
                                   "coupling of the 64 meshes)"},
            "tiles": self.plan.tiles, "tune": self.tuned,
            "plan_s": self.t_plan, "plan_cached_tuning_s": self.t_plan_cached,
            "plan_note": "plan_s includes the autotuner's timed candidates; "
                         "plan_cached_tuning_s is the same plan with the tuning read from its "
                         "cache file",
            "bases_s": self.t_bases,
        }


class LearnedBench:
    """Learned form: the order selector trained on the GPU on 1e6 pairs drawn
    from the near fields of the config-1..3 meshes (the 512-, 8192- and
    32768-triangle spheres and the 24576-triangle cube; Laplace SLP/DLP on
    all, Helmholtz kappa 2/4/8 SLP/DLP on the last two) and 2.4e5 pairs of
    the admissible blocks of the two finer spheres, then applied to the
    near field of a large sphere: selection (FP16 inference) + per-entry
    order assembly against the plain fixed-order assembly."""

    TOL, MARGIN = 1e-7, 0.5
    GROUP = 4  # rows of a column per network evaluation

    def __init__(self, pk, ctx, n):
        import torch
        from bem_inputs import cube_surface, octahedron_sphere
        from paper_1510_07244_amd.selector import Selector, samples
        self.pk, self.ctx = pk, ctx
        L, H = pk.LAPLACE, pk.HELMHOLTZ
        jobs = []
        s1, s2, s3, cube = (octahedron_sphere(8), octahedron_sphere(32), octahedron_sphere(64),
                            cube_surface(32))
        for layer in (0, 1):
            jobs.append((s1.v, s1.tri, pk.make_op(L, layer), 40000, 10 + layer))
            jobs.append((s2.v, s2.tri, pk.make_op(L, layer), 120000, 20 + layer))
            jobs.append((s3.v, s3.tri, pk.make_op(L, layer), 100000, 30 + layer))
            jobs.append((cube.v, cube.tri, pk.make_op(L, layer), 40000, 40 + layer))
            # pairs of the admissible blocks (the coupling blocks' entries)
            jobs.append((s2.v, s2.tri, pk.make_op(L, layer), 60000, 70 + layer, "far"))
            jobs.append((s3.v, s3.tri, pk.make_op(L, layer), 60000, 80 + layer, "far"))
            for k in (2.0, 4.0, 8.0):
                jobs.append((s3.v, s3.tri, pk.make_op(H, layer, kappa=k), 40000, 50 + layer + int(k)))
                jobs.append((cube.v, cube.tri, pk.make_op(H, layer, kappa=k), 26667, 60 + layer + int(k)))
        t0 = time.perf_counter()
        X, T = samples(ctx, jobs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        self.sel = Selector(ctx, seed=0)
        self.sel.set_standardisation(X)
        self.losses = self.sel.fit(X, T, epochs=20, batch=4096, lr=2e-3, seed=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        self.n_train, self.t_samples, self.t_train = int(X.shape[0]), t1 - t0, t2 - t1
        del X, T
        self.m = m = octahedron_sphere(n)
        self.mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
        ct = pk.ClusterTree(m.v, m.tri, leaf=64)
        near, _ = pk.block_tree(ct, eta=2.0)
        self.nblocks = len(near)
        self.near_idx = [(ct.idx(t), ct.idx(s)) for t, s in near]
        self.blocks, self.total = pk.Blocks.from_lists([ct.idx(t) for t, s in near],
                                                       [ct.idx(s) for t, s in near])
        # blocks for the error check (seeded sample), as offsets into the output
        sizes = np.array([ct.idx(t).size * ct.idx(s).size for t, s in near], dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        rng = np.random.Generator(np.random.PCG64(5))
        self.check = [(int(offs[k]), int(sizes[k])) for k in rng.choice(len(near), 256, replace=False)]
        # pair classes of the whole near field (for the rooflines)
        self.counts = class_counts(m.tri, [ct.idx(t) for t, s in near], [ct.idx(s) for t, s in near])

    def leg(self, torch, op, stream, steps, warmup):
        ctx, pk = self.ctx, self.pk
        dt = pk.out_dtype(op)
        plain = torch.empty(self.total, dtype=dt, device="cuda")
        learned = torch.empty(self.total, dtype=dt, device="cuda")
        orders = torch.empty(self.total, dtype=torch.int8, device="cuda")
        sel = lambda g: ctx.select_orders(self.mesh, op, self.blocks, self.sel.params, orders,
                                          self.TOL, self.MARGIN, 2, stream, range=self.sel.range,
                                          group=g)
        runs = {
            "plain": lambda: ctx.assemble_nearfield(self.mesh, op, self.blocks, plain, stream),
            "select_per_entry": lambda: sel(1),
            "select": lambda: sel(self.GROUP),
            "learned": lambda: ctx.assemble_nearfield_learned(self.mesh, op, self.blocks, orders,
                                                              learned, stream),
        }
        ms = {}
        for name in ("plain", "select_per_entry", "select", "learned"):
            for _ in range(warmup):
                runs[name]()
            ctx.check(stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                runs[name]()
            e1.record(stream)
            e1.synchronize()
            ctx.check(stream)
            ms[name] = e0.elapsed_time(e1) / steps
        q = orders.to(torch.int64)
        reg = q > 0
        qp = op.q_regular
        counts = {int(k): int((q == k).sum()) for k in range(2, qp + 1)}
        pts_plain = float(reg.sum()) * qp ** 4
        pts_learned = float((q[reg] ** 4).sum())
        errs = []
        for o, n in self.check:
            a, b = learned[o:o + n], plain[o:o + n]
            errs.append(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)))
        tot = float(torch.linalg.vector_norm(learned - plain) / torch.linalg.vector_norm(plain))
        del plain, learned, orders
        # rooflines of the two assemblies: the model flops of the plain rule,
        # and of the learned orders (regular pairs at their own order, the
        # singular pairs by the same Sauter-Schwab rules)
        F = FLOPS_PER_POINT[(op.kernel, op.layer)]
        f_plain = near_flops(self.counts, op.kernel, op.layer, qp, op.q_singular)
        f_learned = f_plain - float(self.counts[0]) * qp ** 4 * F + \
            sum(float(n) * k ** 4 * F for k, n in counts.items())
        peak = FP64_VALU_PEAK
        roof = lambda f, t: {"bound": "alu", "achieved": f / (t * 1e-3) / 1e12,
                             "peak": peak / 1e12, "unit": "TFLOP/s", "frac": f / (t * 1e-3) / peak,
                             "flops_per_launch": f, "ms_per_launch": t}
        return {"plain_ms": ms["plain"], "select_ms": ms["select"], "learned_ms": ms["learned"],
                "roofline_plain": roof(f_plain, ms["plain"]),
                "roofline_learned": roof(f_learned, ms["learned"]),
                "select_per_entry_ms": ms["select_per_entry"],
                "speedup_vs_plain": ms["plain"] / (ms["select"] + ms["learned"]),
                "assembly_speedup_excl_select": ms["plain"] / ms["learned"],
                "points_fraction": pts_learned / pts_plain, "orders": counts,
                "max_block_rel_err_vs_plain": max(errs), "near_field_rel_err_vs_plain": tot,
                "entries": int(self.total)}

    def result(self, torch, stream, steps, warmup, cpu_seconds=0.0):
        pk = self.pk
        legs = {}
        for name, op in (("laplace_slp", pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)),
                         ("laplace_dlp", pk.make_op(pk.LAPLACE, pk.DLP, q_regular=4, q_singular=4)),
                         ("helmholtz8_slp", pk.make_op(pk.HELMHOLTZ, pk.SLP, q_regular=5,
                                                       q_singular=5, kappa=8.0)),
                         ("helmholtz8_dlp", pk.make_op(pk.HELMHOLTZ, pk.DLP, q_regular=5,
                                                       q_singular=5, kappa=8.0))):
            legs[name] = self.leg(torch, op, stream, steps, warmup)
        if cpu_seconds > 0:
            # the oracle on a seeded sample of the same near-field blocks
            # (Laplace single layer, q = 4, all host threads)
            import oracle
            oracle.use_native_build()
            rng = np.random.Generator(np.random.PCG64(2))
            work = [(*self.near_idx[k], 0) for k in rng.permutation(self.nblocks)]
            n, used, dt = oracle_block_run(self.m, work, cpu_seconds)
            leg = legs["laplace_slp"]
            leg["cpu_oracle"] = {"value": n / dt, "unit": "entries/s",
                                 "cores": oracle.num_threads(), "kind": "oracle",
                                 "sample": f"{used} of {self.nblocks} blocks (seeded order): "
                                           f"{n} entries in {dt:.1f} s",
                                 "gpu_plain_value": leg["entries"] / (leg["plain_ms"] * 1e-3)}
        return {
            "workload": f"near field of the octahedron sphere with {self.m.nt} triangles "
                        f"({self.nblocks} blocks, leaf 64, eta 2): plain fixed order (q=4 Laplace, "
                        "q=5 Helmholtz kappa 8) vs learned per-entry orders "
                        f"(tol {self.TOL}, margin {self.MARGIN}; one network evaluation per "
                        f"run of {self.GROUP} rows of a column, select_per_entry_ms: one per "
                        "entry); FP64",
            "training": {"pairs": self.n_train, "samples_s": self.t_samples,
                         "train_s": self.t_train, "loss_first_epoch": float(self.losses[0]),
                         "loss_last_epoch": float(self.losses[-1])},
            "legs": legs,
        }


def learned_h2_leg(torch, pk, ctx, hb, sel, stream, steps, warmup, tol=1e-7, margin=0.5):
    """The H^2 step with learned orders on the coupling blocks: per entry of
    the single- and double-layer coupling lists the order the selector picks
    (chosen once in the setup), assembled by the per-entry-order kernel (the
    single layer's list unmirrored: that kernel evaluates every block); the
    near field and the bases as in the plain step.  Coupling matrices against
    the plain step's, entry counts and point counts."""
    h, o = hb.h, hb.out
    cs_full, n_cs = h.coupling_blocks(hb.V, hb.V)
    lists = {"cs": (cs_full, n_cs, hb.ops[0]), "cd": (hb.cd, hb.n_cd, hb.ops[1])}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    orders = {k: sel.orders(h.mesh, op, b, n, tol, margin) for k, (b, n, op) in lists.items()}
    torch.cuda.synchronize()
    t_select = time.perf_counter() - t0
    out = {k: torch.empty(n, dtype=torch.float64, device="cuda") for k, (b, n, op) in lists.items()}
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("bases", "nb", "cs", "cd")}
    phase = {k: [] for k in ev}

    def step(record):
        if record:
            ev["bases"][0].record(stream)
        h.basis_replay(hb.V, stream)
        h.basis_replay(hb.W, stream)
        if record:
            ev["bases"][1].record(stream)
            ev["nb"][0].record(stream)
        ctx.assemble_nearfield_both(h.mesh, hb.ops[0], hb.near_s, o["ns"], o["nd"], stream)
        if record:
            ev["nb"][1].record(stream)
        for k, (b, n, op) in lists.items():
            if record:
                ev[k][0].record(stream)
            ctx.assemble_nearfield_learned(h.mesh, op, b, orders[k], out[k], stream)
            if record:
                ev[k][1].record(stream)

    for _ in range(warmup):
        step(False)
    ctx.check(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
        torch.cuda.synchronize()
        for k in ev:
            phase[k].append(ev[k][0].elapsed_time(ev[k][1]))
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.check(stream)
    res = {"ms_per_step": ms, "phase_ms": {k: float(np.mean(v)) for k, v in phase.items()},
           "select_s": t_select, "tol": tol, "margin": margin}
    for k, (b, n, op) in lists.items():
        q = orders[k].to(torch.int64)
        res[k] = {"entries": int(n), "points_fraction": float((q ** 4).sum()) / (n * Q ** 4),
                  "orders": {int(v): int((q == v).sum()) for v in range(2, Q + 1)},
                  "rel_err_vs_plain": float(torch.linalg.vector_norm(out[k] - o[k]) /
                                                torch.linalg.vector_norm(o[k]))}
    res["plain_ms_per_step_one_stream"] = None
    return res


def run_leg(torch, ctx, hb, stream, steps, warmup):
    """Time `steps` steps after `warmup`; per-phase HIP-event means."""
    names = hb.phases
    evs = [{k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for k in names} for _ in range(steps)]
    for _ in range(warmup):
        hb.step(stream)
    ctx.check(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        hb.step(stream, evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check(stream)
    phase = {k: float(np.mean([e[k][0].elapsed_time(e[k][1]) for e in evs])) for k in names}
    return (t1 - t0) * 1e3 / steps, phase


def helmholtz_near_leg(torch, pk, ctx, stream, reps):
    """Near field of the Helmholtz single and double layer (kappa = 4, q = 5,
    complex128) on the 32768-triangle sphere: the one-pass call on the
    mirrored list against the per-layer calls (mirrored single layer, full
    double layer).  Both layers enter the Brakhage-Werner formulation."""
    from paper_1510_07244_amd.h2 import H2Setup
    from bem_inputs import octahedron_sphere
    mh = octahedron_sphere(64)
    h = H2Setup(ctx, mh.v, mh.tri, kernel=pk.HELMHOLTZ, kappa=4.0, q_regular=5, q_singular=5)
    half, total = h.near_blocks(mirror=True)
    full, _ = h.near_blocks()
    c128 = dict(dtype=torch.complex128, device="cuda")
    s, d = torch.empty(total, **c128), torch.empty(total, **c128)
    calls = {
        "one_pass": lambda: ctx.assemble_nearfield_both(h.mesh, h.op(pk.SLP), half, s, d, stream),
        "slp_mirrored": lambda: ctx.assemble_nearfield(h.mesh, h.op(pk.SLP), half, s, stream),
        "dlp": lambda: ctx.assemble_nearfield(h.mesh, h.op(pk.DLP), full, d, stream),
    }
    ms = {}
    for k, call in calls.items():
        call()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            call()
            b.record(stream)
        torch.cuda.synchronize()
        ms[k] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    ctx.check(stream)
    return {"workload": f"Helmholtz kappa 4 SLP + DLP near field, octahedron sphere {mh.nt} "
                        f"triangles ({len(h.near)} blocks, leaf 64, eta 2), q = 5, complex128",
            "entries_per_layer": int(total), "ms": ms,
            "speedup_one_pass": (ms["slp_mirrored"] + ms["dlp"]) / ms["one_pass"]}


def rank_head_leg(torch, pk, ctx, m):
    """The learned rank head: trained on the finished setups of other meshes,
    its caps bound the pivot search of this mesh's bases (searched again
    without the bound where a cap is reached, so the bases are unchanged)."""
    from paper_1510_07244_amd.h2 import H2Setup
    from paper_1510_07244_amd.selector import RankHead, cluster_features
    from bem_inputs import cube_surface, octahedron_sphere, perturbed_sphere

    def setup(mesh):
        h = H2Setup(ctx, mesh.v, mesh.tri, kernel=pk.LAPLACE, q_regular=Q, q_singular=Q)
        return h, h.bases((0, 1))

    train = [setup(x) for x in (octahedron_sphere(16), cube_surface(16), perturbed_sphere(101),
                                perturbed_sphere(102))]
    head = RankHead(ctx, seed=3)
    X, R = RankHead.samples(train)
    t0 = time.perf_counter()
    losses = head.fit(X, R)
    t_train = time.perf_counter() - t0
    h = H2Setup(ctx, m.v, m.tri, kernel=pk.LAPLACE, q_regular=Q, q_singular=Q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = h.bases((0, 1))
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    need = h.needed  # clusters with a basis (the others enter no product)
    err = np.concatenate([np.abs(head.predict(cluster_features(h, B.side)) - B.rank)[need]
                          for B in plain])
    t0 = time.perf_counter()
    caps = [head.caps(h, 0), head.caps(h, 1)]
    t_infer = time.perf_counter() - t0
    t0 = time.perf_counter()
    capped = h.bases((0, 1), rank_caps=caps)
    torch.cuda.synchronize()
    t_capped = time.perf_counter() - t0
    same = all(np.array_equal(a.rank, b.rank) for a, b in zip(plain, capped))
    pinv = lambda Bs: int(sum(lv.cls.size * lv.max_rank ** 2 * 8 for B in Bs for lv in B.levels))
    return {
        "workload": "trained on the setups of a 2048-triangle sphere, a 3072-triangle cube and "
                    "two perturbed spheres (both sides, Laplace, ACA 5e-8); applied to the "
                    f"{m.nt}-triangle sphere's {int(h.needed.sum())} clusters with a basis "
                    "x 2 sides",
        "train_samples": int(R.size), "train_s": t_train,
        "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1]),
        "rank_mean": float(np.mean([B.rank[need].mean() for B in plain])),
        "abs_err_mean": float(err.mean()), "abs_err_max": float(err.max()),
        "cap_margin": 8, "levels": h.cap_stats["levels"], "fallback_levels": h.cap_stats["fallbacks"],
        "pinv_bytes_plain": pinv(plain), "pinv_bytes_capped": pinv(capped),
        "bases_s_plain": t_plain, "bases_s_capped": t_capped, "inference_s": t_infer,
        "bases_equal": bool(same),
    }


def run_concurrent(torch, hb, stream, steps, warmup):
    """Time `steps` concurrent steps after `warmup` (HIP events on the
    joining stream and wall clock)."""
    for _ in range(warmup):
        hb.step_concurrent(torch, stream)
    torch.cuda.synchronize()
    hb.check_concurrent()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(steps):
        hb.step_concurrent(torch, stream)
    b.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hb.check_concurrent()
    return (t1 - t0) * 1e3 / steps, a.elapsed_time(b) / steps


def step_spread(torch, hb, stream, n):
    """min / median / max of n steps timed one by one (HIP events on the
    joining stream), after the bracketed timing."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        hb.step_concurrent(torch, stream)
        b.record(stream)
    torch.cuda.synchronize()
    hb.check_concurrent()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return {"min": ms[0], "median": float(np.median(ms)), "max": ms[-1], "steps": n}


def per_layer_near(torch, hb, stream, reps):
    """HIP-event means of the per-layer near-field passes (mirrored single
    layer, full double layer) that the one-pass call replaces."""
    calls = hb.near_calls(stream)
    out = {}
    for k in ("ns", "nd"):
        calls[k]()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            calls[k]()
            b.record(stream)
        torch.cuda.synchronize()
        out[k] = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    hb.ctx.check(stream)
    return out


def one_pass_flops(ev, tr_, k, q):
    """Near field of both layers in one pass over the mirrored list: per
    evaluated regular pair the double layer's work plus the single layer's
    accumulation (a complex one is two FMAs; the transposed pair's double
    layer costs per-point work only); singular pairs: both layers of (i, j),
    the double layer of (j, i) and the single layer of edge-adjacent
    (j, i)."""
    sing = lambda c: [0] + list(c[1:])
    acc = 2.0 if k == 0 else 4.0
    return (float(ev[0]) * (q * q) ** 2 * (FLOPS_PER_POINT[(k, 1)] + acc) +
            near_flops(sing(ev), k, 0, q, q) + near_flops(sing(ev), k, 1, q, q) +
            near_flops([0, tr_[1], tr_[2], 0], k, 1, q, q) +
            near_flops([0, 0, tr_[2], 0], k, 0, q, q))


def step_flops(hb):
    """Algorithmic flops of the step's block launches (near field of both
    layers in one pass, single-layer coupling on the mirrored list, double-
    layer coupling), by the per-point-pair counts."""
    k, q = hb.kernel, hb.q
    f_nb = one_pass_flops(hb.ev_pairs, hb.tr_pairs, k, q)
    f_cs = float(hb.n_cs // 2) * (q * q) ** 2 * FLOPS_PER_POINT[(k, 0)]
    f_cd = float(hb.n_cd) * (q * q) ** 2 * FLOPS_PER_POINT[(k, 1)]
    return {"nb": f_nb, "cs": f_cs, "cd": f_cd}


def helmholtz_h2_leg(torch, pk, ctx, stream, steps=3, warmup=1, peak64=None, cpu_seconds=0.0):
    """The Helmholtz workloads: SLP + DLP H^2 matrices of the 32768-triangle
    sphere and the 24576-triangle cube surface, kappa 2, 4 and 8, q = 5,
    plain complex128 and mixed complex64: setup time (trees, bases with the
    host pivot search, first assembly) and the step on one stream (bases
    replay, one-pass near field, both couplings) with per-phase HIP-event
    times and the roofline of the longest launch.  With cpu_seconds > 0
    the plain kappa = 4 records carry the oracle's rate on a seeded sample
    of the same step's blocks (all host threads, that many seconds)."""
    from bem_inputs import cube_surface, octahedron_sphere
    out = []
    for name, mesh in (("sphere32768", octahedron_sphere(64)), ("cube24576", cube_surface(32))):
        for kappa in (2.0, 4.0, 8.0):
            for mixed in (False, True):
                hb = H2Bench(pk, ctx, mesh, mixed=mixed, kernel=pk.HELMHOLTZ, kappa=kappa, q=5)
                ms, phase = run_leg(torch, ctx, hb, stream, steps, warmup)
                fl = step_flops(hb)
                longest = max(("nb", "cs", "cd"), key=lambda k: phase[k])
                peak = (FP32_VALU_PEAK if mixed else FP64_VALU_PEAK) / 1e12
                ach = fl[longest] / (phase[longest] * 1e-3) / 1e12
                out.append({
                    "mesh": name, "kappa": kappa,
                    "form": "mixed complex64" if mixed else "plain complex128",
                    "h2_setup_s": hb.t_setup, "bases_s": hb.t_bases,
                    "bases_split": dict(hb.h.bases_time), "ms_per_step": ms, "phase_ms": phase,
                    "entries_evaluated_per_step": hb.entries_evaluated(),
                    "value": hb.entries_evaluated() / (ms * 1e-3),
                    "near_blocks": len(hb.h.near), "far_blocks": len(hb.h.far),
                    "roofline": {"launch": {"nb": "one-pass near field", "cs": "SLP coupling",
                                            "cd": "DLP coupling"}[longest],
                                 "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                                 "frac": ach / peak, "flops_per_launch": fl[longest]},
                })
                if cpu_seconds > 0 and kappa == 4.0 and not mixed:
                    out[-1]["cpu_oracle"] = oracle_sample(mesh, hb, cpu_seconds, pk.HELMHOLTZ,
                                                          kappa, 5)
                del hb
    return out


def batched_config2_leg(torch, pk, ctx, hb, stream, steps=10):
    """The batched form on the config-2 matrix: one persistent plan holding
    the whole matrix step (the mirrored near field with both layers in one
    pass, the mirrored single-layer coupling and the double-layer coupling,
    each list with its own layer and sub-tile shape in one cost-sorted
    queue), autotuned, replayed after the bases; setup = the plain setup plus
    the plan (with its tuning cached, as on a second run), outputs against
    the plain step's."""
    h, o = hb.h, hb.out
    out = {k: torch.empty_like(v) for k, v in o.items()}
    entries = [(h.mesh, hb.near_s, out["ns"], 0, pk.BATCH_BOTH, out["nd"]),
               (h.mesh, hb.cs, out["cs"], 1, pk.BATCH_SLP),
               (h.mesh, hb.cd, out["cd"], 1, pk.BATCH_DLP)]
    cache = os.path.join(tempfile.gettempdir(), f"bem_tune_c2_{os.getpid()}.txt")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [pk.Plan(ctx, hb.ops[0], entries, autotune=True, cache=cache, stream=stream)]
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    tuned = [p.config for p in plans]
    for p in plans:
        p.close()
    t0 = time.perf_counter()
    plans = [pk.Plan(ctx, hb.ops[0], entries, autotune=True, cache=cache, stream=stream)]
    torch.cuda.synchronize()
    t_cached = time.perf_counter() - t0
    os.remove(cache)

    # the coupling lists need the pivots only, not the basis matrices: the
    # bases run on a second stream beside the plan (the plan has its own
    # geometry buffer), as the plain step's bases beside its near field
    side = torch.cuda.Stream()

    def step():
        side.wait_stream(stream)
        h.basis_replay(hb.V, side)
        h.basis_replay(hb.W, side)
        for p in plans:
            p.run(stream)
        stream.wait_stream(side)
    step()
    ctx.check(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    e1.synchronize()
    ctx.check(stream)
    ms = e0.elapsed_time(e1) / steps
    hb.step(stream)  # the plain step's outputs, for the comparison
    torch.cuda.synchronize()
    diff = {k: float(torch.linalg.vector_norm(out[k] - o[k]) / torch.linalg.vector_norm(o[k]))
            for k in out}
    for p in plans:
        p.close()
    return {"value": hb.entries_evaluated() / (ms * 1e-3), "unit": "entries/s",
            "ms_per_step": ms, "plan_tuning_s": t_tune, "plan_cached_tuning_s": t_cached,
            "h2_setup_s": float(hb.t_setup) + t_cached, "tune": tuned,
            "rel_diff_vs_plain_step": diff,
            "note": "one persistent graph replay (near field of both layers in one pass, "
                    "single- and double-layer coupling, one queue) beside the bases on a "
                    "second stream"}


def solve_leg(torch, pk, ctx, hb, stream, reps=20):
    """H^2 products with the step's assembled matrices (near field, coupling
    and nested bases; the library's grouped matrix-vector kernels) and the
    interior Dirichlet problem of the paper's Laplace experiment for
    f1 = x1^2 - x3^2: V alpha = (1/2 M + K) beta by conjugate gradients.
    Roofline of the product: bytes of the matrices read once per product
    (near-field entries, coupling entries, transfer matrices) over its time,
    against HBM."""
    from paper_1510_07244_amd.h2mv import GraphedMatvec, H2Matrix, cg, cg_device
    h, o, m = hb.h, hb.out, hb.m
    Hv = H2Matrix(h, hb.V, hb.V, o["ns"], o["cs"])
    Hk = H2Matrix(h, hb.V, hb.W, o["nd"], o["cd"])
    c = m.v[m.tri].mean(axis=1)
    beta = torch.from_numpy(c[:, 0] ** 2 - c[:, 2] ** 2).cuda()
    y = torch.empty_like(beta)
    res = {}
    def median_ms(f):
        f()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            f()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    for name, H in (("slp", Hv), ("dlp", Hk)):
        eager = median_ms(lambda: H.matvec(beta, y, stream))
        G = GraphedMatvec(H)
        ms = median_ms(lambda: G(beta, y, stream))
        nbytes = 8 * (H.near.numel() + H.coupling.numel() +
                      sum(lv.V.numel() for lv in H.V.levels) +
                      (sum(lv.V.numel() for lv in H.W.levels) if H.W is not H.V else 0))
        res[name] = {"ms_per_product": ms, "eager_ms_per_product": eager, "matrix_bytes": nbytes,
                     "roofline": {"bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                                  "peak": 8000.0, "unit": "GB/s",
                                  "frac": nbytes / (ms * 1e-3) / 8e12},
                     "launches": 1 + len(H.near_calls) + len(H.fwd) + len(H.bwd),
                     "note": "ms_per_product: one replay of the product captured in a HIP graph "
                             "(near field on a second stream); eager: the same launches one by "
                             "one from the host"}
    rhs = torch.empty_like(beta)
    Hk.matvec(beta, rhs, stream)
    ctx.mass_apply(h.mesh, 0.5, beta, rhs, stream)
    alpha_h = torch.zeros_like(beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_h, _ = cg(ctx, GraphedMatvec(Hv), rhs, alpha_h, tol=1e-8, maxit=1000, stream=stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t0
    # every step on the device (the step captured in a HIP graph, the host
    # reads the stopping flag every 8 steps; capture included in the timed
    # call, after one warm-up call)
    cg_device(ctx, Hv, rhs, torch.zeros_like(beta), tol=1e-8, maxit=1000, stream=stream)
    alpha = torch.zeros_like(beta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, rel = cg_device(ctx, Hv, rhs, alpha, tol=1e-8, maxit=1000, stream=stream)
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t0
    x = c / np.linalg.norm(c, axis=1)[:, None]
    dn = 2 * x[:, 0] ** 2 - 2 * x[:, 2] ** 2
    a = alpha.cpu().numpy()
    area = 0.5 * np.linalg.norm(np.cross(m.v[m.tri[:, 1]] - m.v[m.tri[:, 0]],
                                         m.v[m.tri[:, 2]] - m.v[m.tri[:, 0]]), axis=1)
    err = float(np.sqrt((area * (a - dn) ** 2).sum() / (area * dn ** 2).sum()))
    ctx.check(stream)
    res["laplace_dirichlet_f1"] = {"cg_iterations": it, "relative_residual": rel,
                                   "solve_s": t_cg, "neumann_l2_rel_err": err,
                                   "solve_s_host_scalars": t_host,
                                   "host_scalars_iterations": it_h,
                                   "note": "solve_s: cg_device (steps captured in a HIP graph, "
                                           "scalars on the device); host_scalars: cg with the "
                                           "graph-captured product and the step scalars read "
                                           "back every step"}
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_block_run(m, work, limit, kernel=0, kappa=0.0, q=Q):
    """The FP64 oracle over a list of (rows, cols, layer) blocks in order
    until `limit` seconds have passed: (entries, blocks, seconds)."""
    import oracle
    n = used = 0
    t0 = time.perf_counter()
    for r, c, layer in work:
        n += oracle.block(m.v, m.tri, r, c, kernel=kernel, kappa=kappa, layer=layer, q_reg=q,
                          q_sing=q).size
        used += 1
        if time.perf_counter() - t0 > limit:
            break
    return n, used, time.perf_counter() - t0


def h2_oracle_work(hb, seed=1):
    """The blocks of an H2 step in a seeded order: near-field blocks and
    coupling blocks (on the pivots), each with both layers."""
    h = hb.h
    rng = np.random.Generator(np.random.PCG64(seed))
    items = [("near", k) for k in range(len(h.near))] + [("far", k) for k in range(len(h.far))]
    work = []
    for idx in rng.permutation(len(items)):
        kind, k = items[idx]
        if kind == "near":
            t, s = h.near[k]
            work += [(h.ct.idx(t), h.ct.idx(s), 0), (h.ct.idx(t), h.ct.idx(s), 1)]
        else:
            t, s = h.far[k]
            work += [(hb.V.piv[t], hb.V.piv[s], 0), (hb.V.piv[t], hb.W.piv[s], 1)]
    return work, len(items)


def oracle_sample(m, hb, seconds, kernel, kappa, q):
    """The oracle's rate (all host threads) on a seeded sample of an H2
    step's blocks, near field and coupling, both layers."""
    import oracle
    oracle.use_native_build()
    work, nitems = h2_oracle_work(hb)
    n, used, dt = oracle_block_run(m, work, seconds, kernel, kappa, q)
    return {"value": n / dt, "unit": "entries/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{(used + 1) // 2} of {nitems} blocks (seeded order), "
                                        f"both layers: {n} entries in {dt:.1f} s"}


def cpu_baseline(m, hb, seconds):
    """The FP64 oracle (built here with -O3 -march=native) on a seeded
    sample of the step's blocks, near field and coupling, both layers: all
    host threads for `seconds`, then one thread for a third of that."""
    import oracle
    oracle.use_native_build()
    work, nitems = h2_oracle_work(hb)

    def run(limit):
        n, used, dt = oracle_block_run(m, work, limit)
        return n, (used + 1) // 2, dt

    threads = oracle.num_threads()
    n, used, dt = run(seconds)
    oracle.set_threads(1)
    n1, used1, dt1 = run(seconds / 3)
    oracle.set_threads(threads)
    return {"value": n / dt, "unit": "entries/s", "cores": threads, "kind": "oracle",
            "sample": f"{used} of {nitems} blocks (near field and coupling, seeded order), SLP "
                      f"and DLP each: {n} entries in {dt:.1f} s on {threads} threads",
            "one_thread": {"value": n1 / dt1, "sample": f"first {used1} blocks of the same "
                                                        f"order: {n1} entries in {dt1:.1f} s"},
            "build": "gcc -O3 -march=native -fopenmp (compiled on this host)",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): block assembly shards "
              "over GPUs without communication; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1510_07244_amd as pk
    from bem_inputs import octahedron_sphere

    m = octahedron_sphere(32)
    ctx = pk.Context(0)
    if args.counter_pass:
        counter_pass(torch, pk, ctx, m)
        return
    setups, bases_split = [], []
    hb = None
    for _ in range(max(1, args.setup_repeats)):
        hb = H2Bench(pk, ctx, m)
        setups.append((hb.t_setup, hb.t_tree, hb.t_bases, hb.t_assembly))
        bases_split.append(dict(hb.h.bases_time))
    stream = torch.cuda.current_stream()
    peak_meas = {"fp64": ctx.valu_peak(True), "fp32": ctx.valu_peak(False)}
    # per-phase timings from the sequential step; the step time from the
    # same step with its independent phases on four streams
    ms_seq, phase = run_leg(torch, ctx, hb, stream, args.steps, args.warmup)
    per_layer = per_layer_near(torch, hb, stream, max(5, min(args.steps, 20)))
    if args.one_stream:
        ms_step, ms_step_ev = ms_seq, ms_seq
        spread = None
    else:
        ms_step, ms_step_ev = run_concurrent(torch, hb, stream, args.steps, args.warmup)
        spread = step_spread(torch, hb, stream, max(5, min(args.steps, 10)))
    hm = H2Bench(pk, ctx, m, mixed=True)
    ms_seq_m, phase_m = run_leg(torch, ctx, hm, stream, args.steps, args.warmup)
    ms_step_m = ms_seq_m if args.one_stream else run_concurrent(torch, hm, stream, args.steps,
                                                                 args.warmup)[0]
    solve = solve_leg(torch, pk, ctx, hb, stream)
    batched_c2 = None if args.batched_meshes <= 0 else batched_config2_leg(torch, pk, ctx, hb,
                                                                           stream)
    # mixed + batched: the same plan with the mixed operator (FP32 regular
    # pairs, lists with pair lists everywhere), against the mixed step
    batched_c2m = None if args.batched_meshes <= 0 else batched_config2_leg(torch, pk, ctx, hm,
                                                                            stream)
    helmholtz = None if args.no_helmholtz else helmholtz_near_leg(torch, pk, ctx, stream, 5)
    helmholtz_h2 = None if args.no_helmholtz else helmholtz_h2_leg(
        torch, pk, ctx, stream, cpu_seconds=0.0 if args.no_cpu_baseline else args.cpu_seconds / 3)
    batched = None
    if args.batched_meshes > 0:
        bb = BatchedBench(pk, ctx, args.batched_meshes)
        batched = bb.result(torch, stream, args.steps, args.warmup,
                            cpu_seconds=0.0 if args.no_cpu_baseline else args.cpu_seconds / 3)
        del bb
    learned = None
    if args.learned_n > 0:
        lb = LearnedBench(pk, ctx, args.learned_n)
        lb.GROUP = args.learned_group
        learned = lb.result(torch, stream, min(args.steps, 10), 1,
                            cpu_seconds=0.0 if args.no_cpu_baseline else args.cpu_seconds / 3)
        learned["h2_step"] = learned_h2_leg(torch, pk, ctx, hb, lb.sel, stream,
                                            min(args.steps, 10), 2)
        learned["h2_step"]["plain_ms_per_step_one_stream"] = ms_seq
        del lb
        learned["rank_head"] = rank_head_leg(torch, pk, ctx, m)

    h = hb.h
    rows = [h.ct.idx(t) for t, s in h.near]
    cols = [h.ct.idx(s) for t, s in h.near]
    counts = class_counts(m.tri, rows, cols)
    f_dlp = near_flops(counts, 0, 1, Q, Q)
    f_cd = float(hb.n_cd) * (Q ** 2) ** 2 * FLOPS_PER_POINT[(0, 1)]  # coupling: regular pairs only
    counted_cd = stored_counters()[1]
    f_cs_lap = float(hb.n_cs // 2) * (Q ** 2) ** 2 * FLOPS_PER_POINT[(0, 0)]  # evaluated half
    # the mirrored single layer evaluates the pairs (i, j) of the blocks with
    # t < s and the lower triangles of the blocks (t, t), plus the
    # edge-adjacent transposed pairs (as (j, i))
    counts_s = hb.ev_pairs.copy()
    counts_s[2] += hb.tr_pairs[2]
    f_slp = near_flops(counts_s, 0, 0, Q, Q)
    f_both = one_pass_flops(hb.ev_pairs, hb.tr_pairs, 0, Q)
    st = np.array(setups)
    best = int(np.argmin(st[:, 0]))
    ranks_v = hb.V.rank[hb.V.rank > 0]
    ranks_w = hb.W.rank[hb.W.rank > 0]
    result = {
        "metric": METRIC,
        "value": hb.entries_evaluated() / (ms_step * 1e-3),
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
            "workload": "Laplace SLP+DLP H2 matrix, octahedron sphere 8192 triangles, leaf 64, "
                        "eta 2, Sauter-Schwab q=4, Duffy/Gauss q=4, Green order 4, ACA 5e-8, "
                        "plain FP64",
            "triangles": int(m.nt), "near_blocks": int(len(h.near)), "far_blocks": int(len(h.far)),
            "entries_evaluated_per_step": int(hb.entries_evaluated()),
            "entries_written_per_step": int(hb.entries()),
            "written_entries_per_s": hb.entries() / (ms_step * 1e-3),
            "value_counts": "entries evaluated by the kernels per second (the written count, "
                            "which adds the single layer's mirrored copies, is "
                            "written_entries_per_s); the CPU baseline counts every entry the "
                            "oracle evaluates",
            "single_layer_symmetry": "of each pair of blocks (t, s), (s, t), t != s, of the "
                                     "single layer (near field and coupling) the block with t < s "
                                     "is evaluated, the other written as its transpose (near-field "
                                     "edge-adjacent entries evaluated as (j, i))",
            "near_field": "one pass for both layers over the blocks with t <= s: each point "
                          "pair's distance and reciprocal root serve the single layer of (i, j) "
                          "and the double layer of (i, j) and (j, i)",
            "near_entries_per_operator": int(hb.n_near),
            "coupling_entries": {"slp": int(hb.n_cs), "dlp": int(hb.n_cd)},
            "rank_mean": {"row_basis": float(ranks_v.mean()), "dlp_column_basis": float(ranks_w.mean())},
            "pairs_by_class": {"disjoint": int(counts[0]), "vertex": int(counts[1]),
                               "edge": int(counts[2]), "identical": int(counts[3])},
        },
        "h2_setup_s": {"best": float(st[best, 0]), "median": float(np.median(st[:, 0])),
                       "tree": float(st[best, 1]), "bases": float(st[best, 2]),
                       "bases_split": bases_split[best],
                       "bases_split_note": "device: Green matrices and the previous level's "
                                           "pivot inverses and contractions (waited for before "
                                           "the copy); copy: Green matrices to the host; "
                                           "pivot_search: host cross approximation (pivots only, "
                                           "the pivot blocks are inverted on the device)",
                       "assembly": float(st[best, 3]), "repeats": int(st.shape[0])},
        "phase_ms": phase,
        "step_streams": ("one stream" if args.one_stream else
                         "the step's four independent phases (bases, near field, SLP coupling, "
                         "DLP coupling) on four streams, joined per step; phase_ms from the same "
                         "step run on one stream"),
        "ms_per_step_events": ms_step_ev,
        "step_ms_spread": spread,
        "sequential": {"ms_per_step": ms_seq, "value": hb.entries_evaluated() / (ms_seq * 1e-3)},
        "roofline": {
            "kernel": "k_blocks<Laplace, DLP> coupling (the step's longest launch; "
                      "+ geometry kernel in the same call)",
            "bound": "alu", "achieved": f_cd / (phase["cd"] * 1e-3) / 1e12,
            "peak": FP64_VALU_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": f_cd / (phase["cd"] * 1e-3) / FP64_VALU_PEAK, "traffic": stored_traffic(),
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
            "ms_per_launch": phase["cd"], "flops_per_launch": f_cd,
            "peak_measured": peak_meas["fp64"],
            "frac_of_measured_peak": f_cd / (phase["cd"] * 1e-3) / (peak_meas["fp64"] * 1e12),
            "flops_model": "strict: 19 flops per point pair (the reciprocal root as one)",
            "counted_flops_per_launch": counted_cd,
            "counted_frac_of_measured_peak": (None if counted_cd is None else
                                              counted_cd / (phase["cd"] * 1e-3) /
                                              (peak_meas["fp64"] * 1e12)),
            "counted_note": "FP64 FLOP of the launch from the SQ_INSTS_VALU_*_F64 counters of "
                            "the committed counter pass (64 x (2 FMA + ADD + MUL + TRANS)), null "
                            "once the kernel's sources change",
        },
        "valu_peak_measured_tflops": dict(peak_meas, probe="bem_valu_peak: 8 independent FMA "
                                          "chains per lane, 16 waves per CU, best of 5"),
        "roofline_slp_coupling": {
            "kernel": "k_blocks<Laplace, SLP> coupling, mirrored (blocks with t < s, each also "
                      "written transposed)", "bound": "alu",
            "achieved": f_cs_lap / (phase["cs"] * 1e-3) / 1e12, "peak": FP64_VALU_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": f_cs_lap / (phase["cs"] * 1e-3) / FP64_VALU_PEAK,
            "ms_per_launch": phase["cs"], "flops_per_launch": f_cs_lap,
        },
        "roofline_near_both": {
            "kernel": "k_blocks<Laplace, SLP+DLP> near field, one pass over the blocks with "
                      "t <= s (both layers of (t, s) and (s, t))", "bound": "alu",
            "achieved": f_both / (phase["nb"] * 1e-3) / 1e12, "peak": FP64_VALU_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": f_both / (phase["nb"] * 1e-3) / FP64_VALU_PEAK,
            "ms_per_launch": phase["nb"], "flops_per_launch": f_both,
        },
        "near_per_layer": {
            "ms": per_layer, "one_pass_ms": phase["nb"],
            "speedup": (per_layer["ns"] + per_layer["nd"]) / phase["nb"],
            "roofline_dlp": {
                "kernel": "k_blocks<Laplace, DLP> near field (all blocks)", "bound": "alu",
                "achieved": f_dlp / (per_layer["nd"] * 1e-3) / 1e12,
                "frac": f_dlp / (per_layer["nd"] * 1e-3) / FP64_VALU_PEAK,
                "flops_per_launch": f_dlp},
            "roofline_slp": {
                "kernel": "k_blocks<Laplace, SLP> near field (mirrored: blocks with t <= s)",
                "bound": "alu", "achieved": f_slp / (per_layer["ns"] * 1e-3) / 1e12,
                "frac": f_slp / (per_layer["ns"] * 1e-3) / FP64_VALU_PEAK,
                "flops_per_launch": f_slp},
        },
        "forms": {
            "plain_fp64": {"value": hb.entries_evaluated() / (ms_step * 1e-3),
                           "ms_per_step": ms_step},
            "mixed": {
                "value": hm.entries_evaluated() / (ms_step_m * 1e-3), "ms_per_step": ms_step_m,
                "speedup_vs_plain": ms_step / ms_step_m, "phase_ms": phase_m,
                "sequential_ms_per_step": ms_seq_m,
                "near_singular_ratio": MIXED_RATIO,
                "dtype": "f32 regular pairs, f64 singular/near-singular, f32 out",
                "h2_setup_s": float(hm.t_setup),
                "roofline": {
                    "kernel": "k_blocks<Laplace, DLP, mixed> coupling", "bound": "alu",
                    "achieved": f_cd / (phase_m["cd"] * 1e-3) / 1e12,
                    "peak": FP32_VALU_PEAK / 1e12, "unit": "TFLOP/s",
                    "frac": f_cd / (phase_m["cd"] * 1e-3) / FP32_VALU_PEAK,
                    "ms_per_launch": phase_m["cd"], "flops_per_launch": f_cd,
                    "peak_without_packed_fp32": FP64_VALU_PEAK / 1e12,
                    "frac_without_packed_fp32": f_cd / (phase_m["cd"] * 1e-3) / FP64_VALU_PEAK,
                    "peak_measured": peak_meas["fp32"],
                    "frac_of_measured_peak": f_cd / (phase_m["cd"] * 1e-3) /
                                             (peak_meas["fp32"] * 1e12),
                    "note": "the build does not use packed FP32 instructions, whose pairs of "
                            "operations make the 157.3 TFLOP/s figure; without them the FP32 "
                            "vector rate is that of FP64, 78.6",
                },
            },
        },
    }
    result["h2_products"] = solve
    if helmholtz:
        result["forms"]["helmholtz_near_both"] = helmholtz
    if helmholtz_h2:
        result["helmholtz_h2"] = helmholtz_h2
    if batched:
        result["forms"]["batched"] = batched
    if batched_c2:
        result["forms"]["batched_config2"] = batched_c2
    if batched_c2m:
        batched_c2m["speedup_vs_plain"] = ms_step / batched_c2m["ms_per_step"]
        batched_c2m["note"] = ("mixed operator: " + batched_c2m["note"] +
                               "; rel_diff against the mixed step's outputs")
        result["forms"]["mixed_batched_config2"] = batched_c2m
    if learned:
        result["forms"]["learned"] = learned
    # H2 setup time of the 8192-sphere matrix by form (tree, bases, first
    # assembly; the learned form adds the order selection of its coupling
    # lists, the network being trained once offline)
    by_form = {"plain_fp64": float(st[best, 0]), "mixed": float(hm.t_setup)}
    if batched_c2:
        by_form["batched"] = float(st[best, 0]) + batched_c2["plan_cached_tuning_s"]
    if batched_c2m:
        by_form["mixed_batched"] = float(hm.t_setup) + batched_c2m["plan_cached_tuning_s"]
    if learned:
        by_form["learned_coupling"] = float(st[best, 0]) + learned["h2_step"]["select_s"]
    result["h2_setup_s_by_form"] = by_form
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(m, hb, args.cpu_seconds)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
