"""Seeded random index samples (PCG64)."""
import numpy as np


def sample_pairs(nt: int, count: int, seed: int):
    """``count`` uniformly random (row, col) triangle pairs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.integers(0, nt, size=count, dtype=np.int64).astype(np.int32)
    c = rng.integers(0, nt, size=count, dtype=np.int64).astype(np.int32)
    return r, c


def sample_subset(items, count: int, seed: int):
    """``count`` distinct items (or all of them), in their original order."""
    items = np.asarray(items)
    if count >= items.shape[0]:
        return items.copy()
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = np.sort(rng.choice(items.shape[0], size=count, replace=False))
    return items[pick]
