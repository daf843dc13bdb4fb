"""Seeded inputs with many rows whose exact distances to a query are equal
but whose FP64 sums round differently with the order of the terms.

A base row is copied COPIES times, each copy with its coordinates permuted
within groups of coordinates on which every query is constant, so that the
exact distance (a sum over the coordinates) is the same for every copy.  The
row's coordinates span several binades (and for IP the groups' query values
span more), so FP64 partial sums round and the rounded value depends on the
order of the terms.  The other rows are far from every query.  Holds none of
the method's arithmetic: only the random draws."""

import numpy as np

N, D, COPIES = 20000, 128, 150


def planted(metric_l2: bool, B: int, seed: int):
    """(x float32 [N, D], attr int32 [1, N], q float32 [B, D], copy row ids).
    Every copy has attribute 0; the other rows 0 or 1."""
    rng = np.random.default_rng(seed)
    groups, step, spread_binades = (1, 0, 8) if metric_l2 else (4, 8, 8)
    gsize = D // groups
    grp = np.arange(D) // gsize
    mag = np.ldexp(1.0, -step * np.arange(groups))
    spread = np.ldexp(1.0, -rng.integers(0, spread_binades + 1, D).astype(np.int64))
    if metric_l2:
        c = (1.0 + rng.random(groups)) * mag * 0.5
        q = (c[None, :] * (1.0 + 1e-3 * rng.standard_normal((B, groups))))[:, grp]
        base = mag[grp] * spread * rng.choice([-1.0, 1.0], D) * (1.0 + rng.random(D))
        other = rng.standard_normal((N, D)) + 5.0
    else:
        q = ((1.0 + rng.random((B, groups))) * mag)[:, grp]
        base = (1.0 + rng.random(D)) * spread * 4.0
        other = 0.05 * rng.standard_normal((N, D))
    q = q.astype(np.float32)
    x = other.astype(np.float32)
    base = base.astype(np.float32)
    pos = np.sort(rng.choice(N, COPIES, replace=False))
    for p in pos:
        perm = np.arange(D)
        for g in range(groups):
            sl = slice(g * gsize, (g + 1) * gsize)
            perm[sl] = rng.permutation(perm[sl])
        x[p] = base[perm]
    a = rng.integers(0, 2, (1, N)).astype(np.int32)
    a[0, pos] = 0
    return x, a, q, pos
