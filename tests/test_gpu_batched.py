"""GPU tests of the batched persistent form (bem_plan_batched / bem_run_batched).

* Entries of every batch entry equal, bit for bit, those of the per-call
  entry points at the same x-point chunk (the default), for near-field and
  coupling lists of meshes of uneven size, plain and mixed precision,
  Laplace and Helmholtz.
* Graph replays: outputs are overwritten with NaN by eager work between
  replays; every replay reproduces the eager result exactly.
* Against the oracle: sampled blocks at 1e-12 relative (plain FP64).
* The autotuner: a valid configuration, results within rounding of the
  default plan's, and a second plan served from the cache file.
* One plan holding the whole matrix step of an H2 setup (near field of both
  layers in one pass, single- and double-layer coupling, each list with its
  own layer and sub-tile shape): every output equals the per-call bits.
* Host-visible errors (an out-of-range triangle id, invalid layer choices)
  are rejected at plan time; a corrupt tuning cache is ignored; device
  allocation failures forced from the host (BEM_FAULT_INJECT=alloc) are
  reported as BEM_ENOMEM and leave the context usable.
"""
import json

import numpy as np
import pytest

import oracle
from bem_inputs import perturbed_sphere, sample_subset
from oracle import htree

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import paper_1510_07244_amd as pk
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    c = pk.Context(0)
    yield c
    c.close()


def _lists(m, seed, n_near, n_coup):
    cl = htree.cluster_tree(m.v, m.tri, 64)
    near, far = htree.block_tree(cl, 2.0)
    pick = [near[k] for k in sample_subset(np.arange(len(near)), n_near, seed=seed)]
    pick += [b for b in near if b[0] == b[1]][:2]
    nrows = [cl[t].idx for t, s in pick]
    ncols = [cl[s].idx for t, s in pick]
    fk = sample_subset(np.arange(len(far)), n_coup, seed=seed + 1)
    crows = [sample_subset(cl[far[k][0]].idx, 17 + 7 * (k % 5), seed=k) for k in fk]
    ccols = [sample_subset(cl[far[k][1]].idx, 9 + 11 * (k % 4), seed=k + 3) for k in fk]
    return (nrows, ncols), (crows, ccols)


@pytest.fixture(scope="module")
def batch(pk):
    """Four perturbed spheres of uneven size, one near-field and one coupling
    list each (eight batch entries)."""
    import torch
    meshes, entries = [], []
    for seed in (3, 11, 20, 41):
        m = perturbed_sphere(seed, n_min=8, n_max=20)
        mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
        (nr, nc), (cr, cc) = _lists(m, seed, 6, 5)
        for coupling, (rows, cols) in ((0, (nr, nc)), (1, (cr, cc))):
            blocks, total = pk.Blocks.from_lists(rows, cols)
            entries.append(dict(m=m, mesh=mesh, blocks=blocks, total=total, coupling=coupling,
                                rows=rows, cols=cols))
        meshes.append(m)
    return entries


def _per_call(pk, ctx, op, e):
    import torch
    out = torch.full((e["total"],), float("nan"), dtype=pk.out_dtype(op), device="cuda")
    f = ctx.assemble_coupling if e["coupling"] else ctx.assemble_nearfield
    f(e["mesh"], op, e["blocks"], out)
    ctx.check()
    return out


def _plan(pk, ctx, op, batch, **kw):
    import torch
    outs = [torch.full((e["total"],), float("nan"), dtype=pk.out_dtype(op), device="cuda")
            for e in batch]
    plan = pk.Plan(ctx, op, [(e["mesh"], e["blocks"], o, e["coupling"]) for e, o in zip(batch, outs)],
                   **kw)
    return plan, outs


def _bits(t):
    import torch
    x = t.cpu()
    if x.is_complex():
        x = torch.view_as_real(x)
    return x.numpy().view(np.uint8)


def _kw(op):
    return dict(kernel=op.kernel, layer=op.layer, kappa=op.kappa, rule=op.regular_rule,
                q_reg=op.q_regular, q_sing=op.q_singular)


@pytest.mark.parametrize("kernel,layer,precision,kappa", [
    (0, 0, 0, 0.0), (0, 1, 0, 0.0), (0, 0, 1, 0.0), (0, 1, 1, 0.0), (1, 0, 0, 4.0), (1, 1, 1, 4.0)])
def test_batched_equals_per_call_bitwise(pk, ctx, batch, kernel, layer, precision, kappa):
    op = pk.make_op(kernel, layer, precision=precision, q_regular=4, q_singular=4, kappa=kappa,
                    near_singular_ratio=0.5 if precision else 0.0)
    ref = [_per_call(pk, ctx, op, e) for e in batch]
    plan, outs = _plan(pk, ctx, op, batch)
    assert plan.tiles > 0
    plan.run()
    ctx.check()
    for e, r, o in zip(batch, ref, outs):
        assert np.array_equal(_bits(o), _bits(r)), (e["m"].name, e["coupling"])
    plan.close()


def test_graph_replays_match_eager(pk, ctx, batch):
    import torch
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    ref = [_per_call(pk, ctx, op, e) for e in batch]
    plan, outs = _plan(pk, ctx, op, batch)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))  # eager work between replays
        torch.cuda.synchronize()
        plan.run()
        ctx.check()
        for r, o in zip(ref, outs):
            assert np.array_equal(_bits(o), _bits(r)), rep
    plan.close()


def test_batched_against_oracle(pk, ctx, batch):
    op = pk.make_op(pk.LAPLACE, pk.DLP, q_regular=4, q_singular=4)
    plan, outs = _plan(pk, ctx, op, batch)
    plan.run()
    ctx.check()
    for e, o in zip(batch[:4], outs[:4]):
        res = o.cpu().numpy()
        off = 0
        for k, (r, c) in enumerate(zip(e["rows"], e["cols"])):
            g = res[off:off + len(r) * len(c)].reshape(len(c), len(r)).T
            off += len(r) * len(c)
            if k % 3:
                continue
            ref = oracle.block(e["m"].v, e["m"].tri, r, c, **_kw(op)).real
            assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()
    plan.close()


def test_autotune_and_cache(pk, ctx, batch, tmp_path):
    import torch
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    base, base_outs = _plan(pk, ctx, op, batch)
    base.run()
    ctx.check()
    cache = str(tmp_path / "tune.jsonl")
    plan, outs = _plan(pk, ctx, op, batch, autotune=True, cache=cache)
    cfg = plan.config
    assert cfg["tuned_ms"] > 0
    assert 1 <= cfg["tile_rows"] <= 64 and 1 <= cfg["tile_cols"] <= 64
    assert cfg["x_chunk"] in (4, 5, 7, 8, 9) and cfg["grid"] > 0
    for o in outs:
        o.fill_(float("nan"))
    plan.run()
    ctx.check()
    for a, b in zip(base_outs, outs):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    lines = [json.loads(l) for l in open(cache)]
    assert len(lines) == 1 and lines[0]["x_chunk"] == cfg["x_chunk"]
    again, outs2 = _plan(pk, ctx, op, batch, autotune=True, cache=cache)
    c2 = again.config
    assert c2["tuned_ms"] == 0.0  # served from the cache, nothing timed
    assert [c2[k] for k in ("grid", "tile_rows", "tile_cols", "x_chunk")] == \
        [cfg[k] for k in ("grid", "tile_rows", "tile_cols", "x_chunk")]
    assert len(open(cache).readlines()) == 1
    for p in (base, plan, again):
        p.close()
    torch.cuda.synchronize()


def test_autotune_entry_point_fills_the_cache(pk, ctx, batch, tmp_path):
    # bem_autotune times the candidates and keeps no plan; a plan made with
    # the same cache afterwards takes the tuned configuration without timing
    import torch
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    outs = [torch.zeros(e["total"], dtype=torch.float64, device="cuda") for e in batch]
    cache = str(tmp_path / "tune.jsonl")
    cfg = pk.autotune(ctx, op, [(e["mesh"], e["blocks"], o, e["coupling"])
                                for e, o in zip(batch, outs)], cache=cache)
    assert cfg["tuned_ms"] > 0 and cfg["grid"] > 0
    assert len(open(cache).readlines()) == 1
    plan, outs2 = _plan(pk, ctx, op, batch, autotune=True, cache=cache)
    c2 = plan.config
    assert c2["tuned_ms"] == 0.0
    assert [c2[k] for k in ("grid", "tile_rows", "tile_cols", "x_chunk", "granularity")] == \
        [cfg[k] for k in ("grid", "tile_rows", "tile_cols", "x_chunk", "granularity")]
    plan.run()
    ctx.check()
    for e, o in zip(batch, outs2):
        ref = _per_call(pk, ctx, op, e).cpu().numpy()
        got = o.cpu().numpy()
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    plan.close()


@pytest.mark.parametrize("granularity", [1, 2])
def test_fixed_configuration_and_small_tiles(pk, ctx, batch, granularity):
    # a ragged sub-tile shape and a small grid still give the per-call bits,
    # with whole blocks or single sub-tiles as the queue's work items
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    ref = [_per_call(pk, ctx, op, e) for e in batch]
    plan, outs = _plan(pk, ctx, op, batch, tune=dict(grid=7, tile_rows=24, tile_cols=40,
                                                      granularity=granularity))
    assert plan.config["tile_rows"] == 24 and plan.config["grid"] == 7
    assert plan.config["granularity"] == granularity
    plan.run()
    ctx.check()
    for r, o in zip(ref, outs):
        assert np.array_equal(_bits(o), _bits(r))
    plan.close()


def test_plan_rejects_bad_ids_before_launch(pk, ctx):
    import torch
    m = perturbed_sphere(5, n_min=8, n_max=8)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    rows = [np.arange(10, dtype=np.int32)]
    cols = [np.array([0, 1, m.nt], dtype=np.int32)]  # m.nt is out of range
    blocks, total = pk.Blocks.from_lists(rows, cols)
    out = torch.zeros(total, dtype=torch.float64, device="cuda")
    op = pk.make_op(pk.LAPLACE, pk.SLP)
    with pytest.raises(pk.BemError) as ei:
        pk.Plan(ctx, op, [(mesh, blocks, out, 0)])
    assert ei.value.code == pk.BEM_EINVAL
    # an empty batch is a valid plan that does nothing
    empty = pk.Plan(ctx, op, [])
    assert empty.tiles == 0
    empty.run()
    ctx.check()
    empty.close()


def test_plan_outliving_its_context(pk, batch):
    # destroying the context first releases the plan's device resources; the
    # plan then refuses to run, and destroying it afterwards is safe (no use
    # of the freed context, no HIP error left behind for later calls)
    import torch
    c2 = pk.Context(0)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    outs = [torch.zeros(e["total"], dtype=torch.float64, device="cuda") for e in batch[:2]]
    plan = pk.Plan(c2, op, [(e["mesh"], e["blocks"], o, e["coupling"]) for e, o in zip(batch, outs)])
    plan.run()
    c2.check()
    c2.close()
    with pytest.raises(pk.BemError) as ei:
        plan.run()
    assert ei.value.code == pk.BEM_EINVAL
    plan.close()
    x = torch.ones(1024, device="cuda")
    assert float(x.sum()) == 1024.0
    torch.cuda.synchronize()


def test_batched_mirrored_lists_equal_per_call(pk, ctx):
    # single-layer lists that write the transposed blocks too (near field and
    # coupling of an H2 setup): the persistent form gives the per-call bits
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = perturbed_sphere(41, n_min=16, n_max=16)
    h = H2Setup(ctx, m.v, m.tri, q_regular=4, q_singular=4)
    V = h.basis(0)
    lists = [(h.near_blocks(mirror=True), 0), (h.coupling_blocks(V, V, mirror=True), 1)]
    op = h.op(pk.SLP)
    ref, outs = [], []
    for (blocks, total), coupling in lists:
        r = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
        (ctx.assemble_coupling if coupling else ctx.assemble_nearfield)(h.mesh, op, blocks, r)
        ctx.check()
        ref.append(r)
        outs.append(torch.full((total,), float("nan"), dtype=torch.float64, device="cuda"))
    plan = pk.Plan(ctx, op, [(h.mesh, b, o, c) for ((b, _), c), o in zip(lists, outs)])
    plan.run()
    ctx.check()
    for r, o in zip(ref, outs):
        assert np.all(np.isfinite(r.cpu().numpy()))
        assert np.array_equal(_bits(o), _bits(r))
    plan.close()


@pytest.mark.parametrize("kernel,precision,kappa", [(0, 0, 0.0), (1, 0, 4.0), (0, 1, 0.0), (1, 1, 4.0)])
def test_batched_layers_in_one_plan_equal_per_call(pk, ctx, kernel, precision, kappa):
    # one plan holding the whole matrix step of an H2 setup: the mirrored
    # near field with both layers in one pass, the mirrored single-layer
    # coupling and the double-layer coupling (each list its own layer and
    # sub-tile shape in one queue); every output equals the per-call bits
    import torch
    from paper_1510_07244_amd.h2 import H2Setup
    m = perturbed_sphere(23, n_min=16, n_max=16)
    h = H2Setup(ctx, m.v, m.tri, kernel=kernel, kappa=kappa, q_regular=4, q_singular=4)
    V, W = h.bases((0, 1))
    near, n_near = h.near_blocks(mirror=True)
    cs, n_cs = h.coupling_blocks(V, V, mirror=True)
    cd, n_cd = h.coupling_blocks(V, W)
    ops = [h.op(pk.SLP), h.op(pk.DLP)]
    for op in ops:
        op.precision = precision
        op.near_singular_ratio = 0.5 if precision else 0.0
    dt = dict(dtype=pk.out_dtype(ops[0]), device="cuda")
    nan = float("nan")
    ref = {k: torch.full((n,), nan, **dt) for k, n in
           (("ns", n_near), ("nd", n_near), ("cs", n_cs), ("cd", n_cd))}
    ctx.assemble_nearfield_both(h.mesh, ops[0], near, ref["ns"], ref["nd"])
    ctx.assemble_coupling(h.mesh, ops[0], cs, ref["cs"])
    ctx.assemble_coupling(h.mesh, ops[1], cd, ref["cd"])
    ctx.check()
    out = {k: torch.full_like(v, nan) for k, v in ref.items()}
    # the operator's layer is the double layer: every entry names its own
    plan = pk.Plan(ctx, ops[1], [(h.mesh, near, out["ns"], 0, pk.BATCH_BOTH, out["nd"]),
                                 (h.mesh, cs, out["cs"], 1, pk.BATCH_SLP),
                                 (h.mesh, cd, out["cd"], 1, pk.BATCH_OP_LAYER)])
    for rep in range(2):
        for o in out.values():
            o.fill_(nan)
        plan.run()
        ctx.check()
        for k in ref:
            r = ref[k].cpu()
            assert np.all(np.isfinite(torch.view_as_real(r).numpy() if r.is_complex() else r.numpy()))
            assert np.array_equal(_bits(out[k]), _bits(ref[k])), (k, rep)
    plan.close()


def test_plan_layer_arguments_are_checked(pk, ctx):
    import torch
    m = perturbed_sphere(5, n_min=8, n_max=8)
    mesh = pk.Mesh(torch.from_numpy(m.v), torch.from_numpy(m.tri))
    idx = np.arange(12, dtype=np.int32)
    blocks, total = pk.Blocks.from_lists([idx], [idx])
    a = torch.zeros(total, dtype=torch.float64, device="cuda")
    b = torch.zeros(total, dtype=torch.float64, device="cuda")
    op = pk.make_op(pk.LAPLACE, pk.SLP)
    bad = [[(mesh, blocks, a, 0, pk.BATCH_BOTH)],            # no second output
           [(mesh, blocks, a, 0, pk.BATCH_BOTH, a)],         # the same buffer twice
           [(mesh, blocks, a, 1, pk.BATCH_BOTH, b)],         # both layers of a coupling list
           [(mesh, blocks, a, 0, pk.BATCH_DLP, b)],          # second output of one layer
           [(mesh, blocks, a, 0, 4)]]                        # no such layer code
    for entries in bad:
        with pytest.raises(pk.BemError) as ei:
            pk.Plan(ctx, op, entries)
        assert ei.value.code == pk.BEM_EINVAL
    plan = pk.Plan(ctx, op, [(mesh, blocks, a, 0, pk.BATCH_BOTH, b)])
    plan.run()
    ctx.check()
    ra = torch.zeros_like(a)
    rb = torch.zeros_like(b)
    ctx.assemble_nearfield_both(mesh, op, blocks, ra, rb)
    ctx.check()
    assert np.array_equal(_bits(a), _bits(ra)) and np.array_equal(_bits(b), _bits(rb))
    plan.close()


def test_corrupt_tuning_cache_is_ignored(pk, ctx, batch, tmp_path):
    # a cache file with garbage, a line of this workload's key with missing
    # fields and one with invalid values: the autotuner times the candidates
    # as with no cache and appends a valid line
    import torch
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    first, _ = _plan(pk, ctx, op, batch, autotune=True, cache=str(tmp_path / "ok.jsonl"))
    key = json.loads(open(tmp_path / "ok.jsonl").readline())["key"]
    first.close()
    cache = tmp_path / "bad.jsonl"
    cache.write_text("not json at all\n"
                     '{"key": "%s", "grid": 512}\n'
                     '{"key": "%s", "grid": -3, "tile_rows": 900, "tile_cols": 0, "x_chunk": 6, '
                     '"granularity": 7, "ms": 1.0}\n' % (key, key))
    plan, outs = _plan(pk, ctx, op, batch, autotune=True, cache=str(cache))
    assert plan.config["tuned_ms"] > 0  # timed: nothing usable was cached
    lines = open(cache).read().splitlines()
    assert len(lines) == 4 and json.loads(lines[-1])["key"] == key
    plan.run()
    ctx.check()
    for e, o in zip(batch, outs):
        ref = _per_call(pk, ctx, op, e).cpu().numpy()
        assert np.abs(o.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    plan.close()
    torch.cuda.synchronize()


def test_allocation_failure_forced_from_the_host(pk, batch, monkeypatch):
    # BEM_FAULT_INJECT=alloc makes the library's device allocations fail:
    # a fresh context's first assembly and a plan report BEM_ENOMEM, write
    # nothing and leave the context usable once the variable is gone
    import torch
    c = pk.Context(0)
    op = pk.make_op(pk.LAPLACE, pk.SLP, q_regular=4, q_singular=4)
    e = batch[0]
    out = torch.full((e["total"],), float("nan"), dtype=torch.float64, device="cuda")
    monkeypatch.setenv("BEM_FAULT_INJECT", "alloc")
    with pytest.raises(pk.BemError) as ei:
        c.assemble_nearfield(e["mesh"], op, e["blocks"], out)
    assert ei.value.code == pk.BEM_ENOMEM
    with pytest.raises(pk.BemError) as ei:
        pk.Plan(c, op, [(e["mesh"], e["blocks"], out, 0)])
    assert ei.value.code == pk.BEM_ENOMEM
    torch.cuda.synchronize()
    assert torch.isnan(out).all()
    monkeypatch.delenv("BEM_FAULT_INJECT")
    c.assemble_nearfield(e["mesh"], op, e["blocks"], out)
    c.check()
    ref = _per_call(pk, c, op, e)
    assert np.array_equal(_bits(out), _bits(ref))
    c.close()
