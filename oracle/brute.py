"""Literal brute-force discrete Morse-Smale complex on tiny simplicial complexes.

Test infrastructure: an independent second reading of the paper used to pin the C oracle.
It differs from the oracle on purpose in every step it can:

* the grid triangulation is built as the Kuhn/Freudenthal subdivision of every unit cube
  into the simplices 0 -> e_p1 -> e_p1+e_p2 -> ... for each permutation p of the axes, plus all
  their faces (the oracle uses anchor + direction-chain cell types);
* the discrete Morse function is Equation 1 taken literally: a cell's value is the tuple of
  its vertices' (value, vertex key) pairs sorted in decreasing order, compared
  lexicographically (F = F(G0) + eps^d F(G1) with a symbolic eps), with ties between equal
  values broken by the larger key (Section 4.1, simulation of simplicity);
* pairing follows Section 3.1 literally: P_alpha is the set of cofacets whose *highest* facet
  is alpha, and an unpaired alpha pairs with the member of P_alpha with the smallest value;
* separatrices are traced as V-paths on the resulting pairs.

Cells are frozensets of vertex indices.
"""
from __future__ import annotations

import itertools
from typing import Dict, FrozenSet, List, Sequence, Tuple

import numpy as np

Cell = FrozenSet[int]


def kuhn_complex(shape: Sequence[int]) -> List[List[Cell]]:
    """All simplices of the Kuhn triangulation of a grid with the given (nx, ny[, nz]) size.

    Vertex index = x + nx*(y + ny*z).  Returns cells grouped by dimension."""
    nd = len(shape)
    strides = [1]
    for s in shape[:-1]:
        strides.append(strides[-1] * s)
    tops = set()
    for anchor in itertools.product(*[range(s - 1) for s in shape]):
        for perm in itertools.permutations(range(nd)):
            pt = list(anchor)
            verts = [sum(p * st for p, st in zip(pt, strides))]
            for ax in perm:
                pt[ax] += 1
                verts.append(sum(p * st for p, st in zip(pt, strides)))
            tops.add(frozenset(verts))
    cells: List[set] = [set() for _ in range(nd + 1)]
    for t in tops:
        for k in range(1, nd + 2):
            for sub in itertools.combinations(sorted(t), k):
                cells[k - 1].add(frozenset(sub))
    return [sorted(c, key=lambda s: tuple(sorted(s))) for c in cells]


def explicit_complex(top_cells: Sequence[Sequence[int]]) -> List[List[Cell]]:
    """All faces of the given top simplices."""
    dim = len(top_cells[0]) - 1
    cells: List[set] = [set() for _ in range(dim + 1)]
    for t in top_cells:
        for k in range(1, dim + 2):
            for sub in itertools.combinations(sorted(t), k):
                cells[k - 1].add(frozenset(sub))
    return [sorted(c, key=lambda s: tuple(sorted(s))) for c in cells]


def F(cell: Cell, h, key) -> Tuple:
    """Equation 1 as a tuple: vertices' (value, key) in decreasing order."""
    return tuple(sorted(((float(h[v]), int(key[v])) for v in cell), reverse=True))


def gradient(cells: List[List[Cell]], h, key=None):
    """Returns (pair, critical): pair maps each paired cell to its partner; critical is a list of
    sets of critical cells per dimension."""
    n = len(cells) - 1
    if key is None:
        key = np.arange(len(h))
    cof: Dict[Cell, List[Cell]] = {c: [] for d in range(n + 1) for c in cells[d]}
    for d in range(1, n + 1):
        for t in cells[d]:
            for v in t:
                cof[t - {v}].append(t)
    pair: Dict[Cell, Cell] = {}
    for d in range(n):
        for a in cells[d]:
            if a in pair:
                continue
            P = []
            for b in cof[a]:
                highest = max((b - {v} for v in b), key=lambda s: F(s, h, key))
                if highest == a:
                    P.append(b)
            if P:
                b = min(P, key=lambda s: F(s, h, key))
                assert b not in pair
                pair[a] = b
                pair[b] = a
    crit = [set(c for c in cells[d] if c not in pair) for d in range(n + 1)]
    return pair, crit, cof


def msc(cells: List[List[Cell]], h, key=None):
    """Critical cells per dimension, descending separatrices (vertex paths from both ends of
    every critical edge), ascending separatrices (top-cell paths from every top cofacet of
    every critical (n-1)-cell; a path that leaves through the boundary ends at None)."""
    n = len(cells) - 1
    pair, crit, cof = gradient(cells, h, key)

    def desc(v):
        path = [v]
        cur = frozenset([v])
        while cur in pair:
            e = pair[cur]
            (w,) = tuple(e - cur)
            path.append(w)
            cur = frozenset([w])
        return tuple(path)

    def asc(T):
        path = [T]
        while T in pair:
            tau = pair[T]
            others = [x for x in cof[tau] if x != T]
            if not others:
                return tuple(path), None
            T = others[0]
            path.append(T)
        return tuple(path), T

    dseps = set()
    for e in crit[1]:
        for v in e:
            dseps.add((e, desc(v)))
    aseps = set()
    for s in crit[n - 1]:
        for T in cof[s]:
            p, term = asc(T)
            aseps.add((s, p, term))
    return {"crit": crit, "desc": dseps, "asc": aseps, "pair": pair}


def _edges_of(t: Cell) -> List[Cell]:
    return [frozenset(p) for p in itertools.combinations(sorted(t), 2)]


def connectors(cells: List[List[Cell]], h, key=None, cap: int = 200000):
    """Saddle-saddle connectors of a 3D complex (Section 3.1): every V-path of the 1-2 level from a
    critical triangle (2-saddle) down to a critical edge (1-saddle), enumerated by depth-first
    search as (triangle, edge, triangle, ..., edge) tuples.  A path leaves the level at an edge
    paired with a vertex."""
    pair, crit, _ = gradient(cells, h, key)
    out = set()

    def walk(e, path):
        if len(out) > cap:
            raise RuntimeError("too many connector paths")
        if e in crit[1]:
            out.add(tuple(path + [e]))
            return
        t = pair.get(e)
        if t is None or len(t) != 3:
            return
        for x in _edges_of(t):
            if x != e:
                walk(x, path + [e, t])

    for t0 in crit[2]:
        for e in _edges_of(t0):
            walk(e, [t0])
    return out


def ss_troublemakers(cells: List[List[Cell]], f, g, key=None):
    """Edges where g's 1-2 V-paths from the 2-saddles of f first leave f's: edges reachable from a
    critical triangle of f through edges paired alike in f and g whose own pairing differs."""
    pf, cf, _ = gradient(cells, f, key)
    pg, _, _ = gradient(cells, g, key)
    seen, out = set(), set()
    stack = [e for t in cf[2] for e in _edges_of(t)]
    while stack:
        e = stack.pop()
        if e in seen:
            continue
        seen.add(e)
        if pf.get(e) != pg.get(e):
            out.add(e)
            continue
        t = pf.get(e)
        if t is not None and len(t) == 3:
            stack.extend(x for x in _edges_of(t) if x != e)
    return out
