"""Explains stalls of the correction loop by fp32 floor collisions (test helper, numpy only).

Every edit is a decrease toward the floor lo = smallest fp32 >= f - xi.  Distinct f values can
share a floor where |f - xi| has a larger exponent than f, and at equal values the vertex order
is decided by the vertex id, which can then disagree with f's order.  No decrease can separate
two vertices that are both at their common floor, so such an inverted pair can leave a violation
behind for good (the convergence argument of Section 4.5 assumes exact arithmetic).

A cell's gradient pairing is decided by the lower star of its highest vertex h, i.e. by the order
of the vertices of h's closed 1-ring.  If that order were the same in f and g the cell would be
paired alike in both, so every violation has an order inversion there.  ``explained`` checks the
stronger statement that a stall leaves behind only inversions that are floor collisions: for each
violating cell, some pair of vertices of the closed 1-ring of its highest vertex in f is at its
floor in g, shares that floor, and is ordered by g opposite to f.
"""
from __future__ import annotations

import itertools

import numpy as np


def _chains(ndim: int, d: int):
    """Direction-bit chains 0 < c1 < ... < cd (bitwise inclusion) of the cell types of dimension d,
    in lexicographic order: the cell-id contract of the library interface."""
    full = (1 << ndim) - 1
    out = []
    for ch in itertools.combinations(range(1, full + 1), d):
        if all((ch[i] & ~ch[i + 1]) == 0 for i in range(d - 1)):
            out.append(ch)
    return sorted(out)


def _offsets(c: int, nx: int, ny: int) -> int:
    return (c & 1) + nx * ((c >> 1) & 1) + nx * ny * ((c >> 2) & 1)


def explained(dims, f, g, lo, cells, chunk: int = 1 << 16) -> np.ndarray:
    """dims = (nx, ny, nz); f, g, lo flat fp32 arrays; cells = int64 (k, 2) rows of (dimension,
    cell id).  Returns a bool array: True where the violation has an equal-floor, both-at-floor,
    f/g-inverted pair in the closed 1-ring of the cell's highest vertex in f."""
    nx, ny, nz = dims
    ndim = 2 if nz == 1 else 3
    f = np.asarray(f, np.float32).reshape(-1)
    g = np.asarray(g, np.float32).reshape(-1)
    lo = np.asarray(lo, np.float32).reshape(-1)
    cells = np.asarray(cells, np.int64).reshape(-1, 2)
    full = (1 << ndim) - 1
    # neighbour offsets of the Freudenthal grid: +c and -c for every nonzero c in {0,1}^D
    nbr = []
    for c in range(1, full + 1):
        d = np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])
        nbr.append(d)
        nbr.append(-d)
    ring_d = np.array([[0, 0, 0]] + nbr)                  # (R, 3), slot 0 = the vertex itself
    out = np.zeros(len(cells), dtype=bool)
    pairs = np.array(list(itertools.combinations(range(len(ring_d)), 2)))
    for s in range(0, len(cells), chunk):
        cc = cells[s:s + chunk]
        dim, cid = cc[:, 0], cc[:, 1]
        # highest vertex in f (value, then id) of every cell
        top = np.full(len(cc), -1, np.int64)
        for d in range(ndim + 1):
            sel = dim == d
            if not sel.any():
                continue
            ch = _chains(ndim, d) if d > 0 else [()]
            nt = len(ch)
            a = cid[sel] // nt
            t = cid[sel] % nt
            verts = np.zeros((sel.sum(), d + 1), np.int64)
            verts[:, 0] = a
            for ti, chain in enumerate(ch):
                m = t == ti
                for k, c in enumerate(chain):
                    verts[m, k + 1] = a[m] + _offsets(c, nx, ny)
            fv = f[verts]
            best = verts[:, 0].copy()
            for k in range(1, d + 1):
                w = verts[:, k]
                higher = (fv[:, k] > f[best]) | ((fv[:, k] == f[best]) & (w > best))
                best = np.where(higher, w, best)
            top[sel] = best
        x = top % nx
        y = (top // nx) % ny
        z = top // (nx * ny)
        R = len(ring_d)
        rv = np.zeros((len(cc), R), np.int64)
        ok = np.zeros((len(cc), R), bool)
        for r in range(R):
            X, Y, Z = x + ring_d[r, 0], y + ring_d[r, 1], z + ring_d[r, 2]
            ok[:, r] = (X >= 0) & (X < nx) & (Y >= 0) & (Y < ny) & (Z >= 0) & (Z < nz)
            rv[:, r] = np.where(ok[:, r], X + nx * (Y + ny * Z), 0)
        hit = np.zeros(len(cc), bool)
        for i, j in pairs:
            u, w = rv[:, i], rv[:, j]
            both = ok[:, i] & ok[:, j]
            at_floor = (g[u] == lo[u]) & (g[w] == lo[w]) & (lo[u] == lo[w])
            inv = (f[u] != f[w]) & ((f[u] < f[w]) != (u < w))
            hit |= both & at_floor & inv
        out[s:s + chunk] = hit
    return out


def collision_field(shape, seed: int):
    """A small field built to collide at the floors with xi = 1: most values are multiples of
    2^-30 below 2^-24 (all share the floor -1 + 2^-24, or -1 for 0), the rest multiples of 2^-20
    in [0, 1).  Values are dyadic so g_hat's float64 bound checks stay exact."""
    rng = np.random.default_rng([seed, 31])
    f = (rng.integers(0, 64, size=shape) * 2.0 ** -30).astype(np.float32)
    big = rng.uniform(size=shape) < 0.3
    f[big] = (rng.integers(0, 2 ** 20, size=int(big.sum())) * 2.0 ** -20).astype(np.float32)
    return f, rng
