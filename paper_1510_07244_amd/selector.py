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


def samples(ctx, jobs):
    """Training samples for a list of (mesh arrays v, tri, op, count, seed):
    returns device tensors X (n, 8) and T (n, 6)."""
    import torch
    xs, ts = [], []
    for v, tri, op, count, seed in jobs:
        mesh = Mesh(torch.from_numpy(np.asarray(v)), torch.from_numpy(np.asarray(tri)))
        r, c = near_pairs(v, tri, count, seed)
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

    def set_standardisation(self, X):
        """mu, sigma of the inputs (sigma floored at 1e-3 for constant ones)."""
        import torch
        mu = X.mean(dim=0)
        sd = X.std(dim=0).clamp_min(1e-3)
        self.params[0:8] = mu
        self.params[8:16] = sd
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
        return per_epoch.cpu().numpy()

    def predict(self, X, fp16=True):
        import torch
        y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self.ctx.mlp_forward(self.n_out, self.params, X, y, fp16=fp16)
        return y

    def orders(self, mesh, op, blocks, n_entries, tol, margin, q_min=2, stream=None):
        """int8 order map of the entries of near-field blocks."""
        import torch
        out = torch.zeros(n_entries, dtype=torch.int8, device="cuda")
        self.ctx.select_orders(mesh, op, blocks, self.params, out, tol, margin, q_min, stream)
        return out
