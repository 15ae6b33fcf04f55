"""Learned order selector: training pairs drawn from the near field of given
meshes, samples (inputs and targets) computed by the library, training by
the library's FP32 gradient and Adam kernels, and order maps for near-field
blocks by its FP16 inference.  This module only draws indices, moves arrays
and orders the calls.

Inputs, targets and the decision rule are defined in include/bem.h (learned
order selection).  The network's standardisation (mu, sigma) is set from the
training inputs before training.
"""
import numpy as np

from . import SEL_OUT, Blocks, ClusterTree, Mesh, block_tree, mlp_params
from . import cluster_features as _cluster_features


def near_pairs(v, tri, count, seed, leaf=64, eta=2.0):
    """`count` vertex-disjoint pairs drawn uniformly (seeded PCG64) from the
    entries of the near-field blocks of the mesh's block tree."""
    tri = np.asarray(tri)
    ct = ClusterTree(v, tri, leaf=leaf)
    near, _ = block_tree(ct, eta=eta)
    nr = (ct.end - ct.begin)[near[:, 0]].astype(np.int64)
    nc = (ct.end - ct.begin)[near[:, 1]].astype(np.int64)
    size = nr * nc
    cum = np.cumsum(size)
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, cols, have = [], [], 0
    while have < count:
        k = rng.integers(0, cum[-1], size=2 * (count - have) + 64)
        b = np.searchsorted(cum, k, side="right")
        local = k - (cum[b] - size[b])
        r = ct.perm[ct.begin[near[b, 0]] + local % nr[b]]
        c = ct.perm[ct.begin[near[b, 1]] + local // nr[b]]
        shared = (tri[r][:, :, None] == tri[c][:, None, :]).any(axis=(1, 2))
        r, c = r[~shared], c[~shared]
        take = min(r.size, count - have)
        rows.append(r[:take])
        cols.append(c[:take])
        have += take
    return np.concatenate(rows).astype(np.int32), np.concatenate(cols).astype(np.int32)


def far_pairs(v, tri, count, seed, leaf=64, eta=2.0):
    """`count` pairs drawn uniformly (seeded PCG64) from the entries of the
    admissible blocks of the mesh's block tree (the coupling blocks' pairs
    are a subset of these)."""
    tri = np.asarray(tri)
    ct = ClusterTree(v, tri, leaf=leaf)
    _, far = block_tree(ct, eta=eta)
    nr = (ct.end - ct.begin)[far[:, 0]].astype(np.int64)
    nc = (ct.end - ct.begin)[far[:, 1]].astype(np.int64)
    if far.shape[0] == 0:
        raise ValueError(f"far_pairs: the {tri.shape[0]}-triangle mesh has no admissible "
                         f"blocks at leaf {leaf}, eta {eta}")
    size = nr * nc
    cum = np.cumsum(size)
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.integers(0, cum[-1], size=count)
    b = np.searchsorted(cum, k, side="right")
    local = k - (cum[b] - size[b])
    r = ct.perm[ct.begin[far[b, 0]] + local % nr[b]]
    c = ct.perm[ct.begin[far[b, 1]] + local // nr[b]]
    return r.astype(np.int32), c.astype(np.int32)


def samples(ctx, jobs):
    """Training samples for a list of (mesh arrays v, tri, op, count, seed)
    or (..., seed, "far"): pairs of the near field (default) or of the
    admissible blocks; returns device tensors X (n, 8) and T (n, 6)."""
    import torch
    xs, ts = [], []
    for job in jobs:
        v, tri, op, count, seed = job[:5]
        far = len(job) > 5 and job[5] == "far"
        mesh = Mesh(torch.from_numpy(np.asarray(v)), torch.from_numpy(np.asarray(tri)))
        r, c = (far_pairs if far else near_pairs)(v, tri, count, seed)
        rows = torch.from_numpy(r).cuda()
        cols = torch.from_numpy(c).cuda()
        x = torch.empty((r.size, 8), dtype=torch.float32, device="cuda")
        t = torch.empty((r.size, SEL_OUT), dtype=torch.float32, device="cuda")
        ctx.selector_samples(mesh, op, rows, cols, x, t)
        ctx.check()
        xs.append(x)
        ts.append(t)
    return torch.cat(xs), torch.cat(ts)


class Selector:
    """Network parameters (device FP32) with He-uniform initialisation
    (seeded), trained and applied through the library."""

    def __init__(self, ctx, n_out=SEL_OUT, seed=0):
        import torch
        self.ctx, self.n_out = ctx, n_out
        n = mlp_params(n_out)
        rng = np.random.Generator(np.random.PCG64(seed))
        p = np.zeros(n, dtype=np.float32)
        p[8:16] = 1.0  # sigma
        o = 16
        for n_o, n_i in ((64, 8), (64, 64), (64, 64), (n_out, 64)):
            lim = np.sqrt(6.0 / n_i)
            p[o:o + n_o * n_i] = rng.uniform(-lim, lim, size=n_o * n_i)
            o += n_o * n_i + n_o  # weights, then zero biases
        self.params = torch.from_numpy(p).cuda()
        self.range = None  # set with the standardisation

    def set_standardisation(self, X):
        """mu, sigma of the inputs (sigma floored at 1e-3 for constant ones),
        and the training range (per-input minimum and maximum) outside which
        the order selection keeps the plain rule."""
        import torch
        mu = X.mean(dim=0)
        sd = X.std(dim=0).clamp_min(1e-3)
        self.params[0:8] = mu
        self.params[8:16] = sd
        self.range = torch.cat([X.min(dim=0).values, X.max(dim=0).values]).contiguous()
        torch.cuda.synchronize()

    def fit(self, X, T, epochs=20, batch=4096, lr=2e-3, seed=0, stream=None):
        """Adam on the mean squared error over shuffled mini-batches (the
        learning rate decays linearly to lr / 10).  Returns the mean loss of
        each epoch (read back once at the end)."""
        import torch
        n = X.shape[0]
        P = self.params
        grad = torch.zeros_like(P)
        m = torch.zeros_like(P)
        v = torch.zeros_like(P)
        losses = torch.zeros(epochs * ((n + batch - 1) // batch), dtype=torch.float32, device="cuda")
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        steps = losses.numel()
        step = 0
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                xb = X[idx].contiguous()
                tb = T[idx].contiguous()
                self.ctx.mlp_grad(self.n_out, P, xb, tb, grad, losses[step:step + 1], stream)
                rate = lr * (1.0 - 0.9 * step / max(steps - 1, 1))
                step += 1
                self.ctx.mlp_adam(P, grad, m, v, step, rate, stream=stream)
        per_epoch = losses.view(epochs, -1).mean(dim=1)
        self.adam = (m, v, step)
        return per_epoch.cpu().numpy()

    def save(self, path):
        """bem_mlp_save: parameters, training range and (after fit) Adam's
        moments and step count."""
        m, v, step = getattr(self, "adam", (None, None, 0))
        self.ctx.mlp_save(path, self.n_out, self.params, m, v, range=self.range, step=step)

    def load(self, path, moments=False):
        """bem_mlp_load into this selector (the training range is required;
        moments=True also restores Adam's state)."""
        import torch
        self.range = torch.empty(16, dtype=torch.float32, device="cuda")
        m = v = None
        if moments:
            m, v = torch.empty_like(self.params), torch.empty_like(self.params)
        step = self.ctx.mlp_load(path, self.n_out, self.params, m, v, range=self.range)
        if moments:
            self.adam = (m, v, step)
        return step

    def predict(self, X, fp16=True):
        import torch
        y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self.ctx.mlp_forward(self.n_out, self.params, X, y, fp16=fp16)
        return y

    def orders(self, mesh, op, blocks, n_entries, tol, margin, q_min=2, stream=None,
               guard=True, group=1):
        """int8 order map of the entries of a block list (guard: pairs
        outside the training range keep the plain order; group: rows of a
        column that share one decision)."""
        import torch
        out = torch.zeros(n_entries, dtype=torch.int8, device="cuda")
        self.ctx.select_orders(mesh, op, blocks, self.params, out, tol, margin, q_min, stream,
                               range=self.range if guard else None, group=group)
        return out


# ------------------------------------------------------------ rank head
RANK_SCALE = 100.0  # network output = rank / RANK_SCALE


def cluster_features(h, side):
    """Eight inputs per cluster of an H2 setup `h` for the rank head
    (bem_cluster_features: log2 of its triangle count, log10 of its box
    diagonal, the box's middle and smallest extent over its largest, its
    height in the tree, kappa times the diagonal, the side (0 rows, 1
    double-layer columns), log10 of the pivot-search tolerance)."""
    ct = h.ct
    return _cluster_features(ct.box, ct.begin[:ct.n], ct.end[:ct.n], h.height, h.kappa, side,
                             h.eps)


class RankHead:
    """Per-cluster prediction of the cross approximation's rank at the setup
    tolerance: the selector network with one output, trained on the ranks
    of finished setups by the library's FP32 kernels and run in FP16.  Its
    caps bound the pivot search of H2Setup.bases (which searches again
    without the bound wherever it is reached)."""

    def __init__(self, ctx, seed=0):
        self.net = Selector(ctx, n_out=1, seed=seed)

    @staticmethod
    def samples(items):
        """(h, bases) pairs of finished setups -> inputs (n, 8), ranks (n,)."""
        X, R = [], []
        for h, Bs in items:
            for B in Bs:
                keep = h.needed
                X.append(cluster_features(h, B.side)[keep])
                R.append(B.rank[keep].astype(np.float32))
        return np.concatenate(X), np.concatenate(R)

    def fit(self, X, ranks, epochs=300, batch=256, lr=3e-3, seed=0):
        import torch
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        Td = torch.from_numpy((ranks / RANK_SCALE).astype(np.float32)[:, None]).cuda()
        self.net.set_standardisation(Xd)
        return self.net.fit(Xd, Td, epochs=epochs, batch=batch, lr=lr, seed=seed)

    def predict(self, X):
        import torch
        y = self.net.predict(torch.from_numpy(np.ascontiguousarray(X)).cuda(), fp16=True)
        return y.cpu().numpy()[:, 0] * RANK_SCALE

    def caps(self, h, side, margin=8):
        """Rank caps of every cluster of `h` on one side: prediction + margin."""
        p = self.predict(cluster_features(h, side))
        return np.clip(np.ceil(p + margin), 1, 2 * h.m).astype(np.int64)
