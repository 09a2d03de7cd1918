"""Python access to the plain C oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use
this package.  The product path (``paper_2409_17346_amd``) never imports it.

``build()`` compiles ``dmt_oracle.c`` with gcc into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "dmt_oracle.c")

# Directed rounding modes are used for the floors, so the compiler must honour the dynamic
# rounding mode and never fuse or reassociate floating-point expressions.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-frounding-math", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, "-o", SO, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return SO


_lib = None
P64 = C.POINTER(C.c_int64)
PF = C.POINTER(C.c_float)
P8 = C.POINTER(C.c_uint8)
P32 = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        build()
    L = C.CDLL(SO)
    L.ocx_grid.restype = C.c_void_p
    L.ocx_grid.argtypes = [C.c_int64, C.c_int64, C.c_int64, P64]
    L.ocx_explicit.restype = C.c_void_p
    L.ocx_explicit.argtypes = [C.c_int, C.c_int64, P64, P32, P32, P32]
    L.ocx_free.argtypes = [C.c_void_p]
    L.ocx_top.argtypes = [C.c_void_p]
    L.ocx_ncell.restype = C.c_int64
    L.ocx_ncell.argtypes = [C.c_void_p, C.c_int]
    L.ocx_exists.argtypes = [C.c_void_p, C.c_int, C.c_int64]
    L.ocx_cell_vertices.argtypes = [C.c_void_p, C.c_int, C.c_int64, P32]
    L.oracle_gradient.argtypes = [C.c_void_p, PF, P64 * 4, P64 * 4]
    L.oracle_msc.restype = C.c_void_p
    L.oracle_msc.argtypes = [C.c_void_p, PF]
    L.omsc_count.restype = C.c_int64
    L.omsc_count.argtypes = [C.c_void_p, C.c_int]
    L.omsc_copy.argtypes = [C.c_void_p, C.c_int, P64]
    L.omsc_free.argtypes = [C.c_void_p]
    L.oracle_bounds.argtypes = [PF, C.c_int64, C.c_float, PF, PF]
    L.oracle_correct.restype = C.c_int
    L.oracle_correct.argtypes = [C.c_void_p, PF, PF, C.c_float, C.c_int, C.c_int, C.c_int, C.c_int64,
                                 PF, P8, P64, P64, C.c_int64]
    L.oracle_decode.argtypes = [PF, P8, C.c_int64, P64, PF, C.c_int64, C.c_float, C.c_int, PF]
    L.oracle_residual.restype = C.c_int64
    L.oracle_residual.argtypes = [C.c_void_p, PF, PF, C.c_int, C.c_int, P64, P64, C.c_int64]
    _lib = L
    return L


def _p(a, t):
    return a.ctypes.data_as(t)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32).reshape(-1)


class Complex:
    """An explicit simplicial complex owned by the C oracle."""

    def __init__(self, handle, dims=None):
        self.h = handle
        self.dims = dims
        L = lib()
        self.top = L.ocx_top(handle)
        self.ncell = [L.ocx_ncell(handle, d) for d in range(self.top + 1)]
        self.nv = self.ncell[0]

    @classmethod
    def grid(cls, nx: int, ny: int, nz: int = 1, key=None):
        k = None
        if key is not None:
            key = np.ascontiguousarray(key, dtype=np.int64).reshape(-1)
            k = _p(key, P64)
        h = lib().ocx_grid(nx, ny, nz, k)
        if not h:
            raise ValueError("invalid grid")
        return cls(h, (nx, ny, nz))

    @classmethod
    def explicit(cls, top: int, nv: int, edges=(), tris=(), tets=()):
        arrs = [np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1)) for x in (edges, tris, tets)]
        n = np.array([nv, len(arrs[0]) // 2, len(arrs[1]) // 3, len(arrs[2]) // 4], dtype=np.int64)
        h = lib().ocx_explicit(top, nv, _p(n, P64), _p(arrs[0], P32), _p(arrs[1], P32), _p(arrs[2], P32))
        if not h:
            raise ValueError("invalid complex")
        c = cls(h)
        c._keep = arrs
        return c

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ocx_free(self.h)
            self.h = None

    def exists(self, d: int) -> np.ndarray:
        L = lib()
        return np.array([L.ocx_exists(self.h, d, i) for i in range(self.ncell[d])], dtype=bool)

    def vertices(self, d: int, cid: int):
        out = np.zeros(d + 1, dtype=np.int32)
        if lib().ocx_cell_vertices(self.h, d, int(cid), _p(out, P32)) != 0:
            return None
        return tuple(int(x) for x in out)


def gradient(cx: Complex, h):
    h = _f32(h)
    up = [np.zeros(max(1, cx.ncell[d] if d <= cx.top else 1), dtype=np.int64) for d in range(4)]
    dn = [np.zeros(max(1, cx.ncell[d] if d <= cx.top else 1), dtype=np.int64) for d in range(4)]
    UA = (P64 * 4)(*[_p(a, P64) for a in up])
    DA = (P64 * 4)(*[_p(a, P64) for a in dn])
    lib().oracle_gradient(cx.h, _p(h, PF), UA, DA)
    return up[:cx.top + 1], dn[:cx.top + 1]


@dataclass
class MSC:
    crit: list
    desc_saddle: np.ndarray
    desc_offsets: np.ndarray
    desc_cells: np.ndarray
    desc_terminal: np.ndarray
    asc_saddle: np.ndarray
    asc_offsets: np.ndarray
    asc_cells: np.ndarray
    asc_terminal: np.ndarray
    min_label: np.ndarray
    max_label: np.ndarray


def msc(cx: Complex, h) -> MSC:
    L = lib()
    h = _f32(h)
    m = L.oracle_msc(cx.h, _p(h, PF))

    def get(what):
        n = L.omsc_count(m, what)
        out = np.zeros(max(n, 0), dtype=np.int64)
        if n > 0:
            L.omsc_copy(m, what, _p(out, P64))
        return out
    try:
        return MSC([get(d) for d in range(cx.top + 1)], get(10), get(11), get(12), get(13),
                   get(20), get(21), get(22), get(23), get(30), get(31))
    finally:
        L.omsc_free(m)


def _separatrices(saddle, offsets, cells, terminal) -> dict:
    """{(saddle, first cell): (terminal, cell sequence)} for one branch family."""
    out = {}
    for b in range(len(saddle)):
        seq = tuple(int(x) for x in cells[offsets[b]:offsets[b + 1]])
        out[(int(saddle[b]), seq[0] if seq else -1)] = (int(terminal[b]), seq)
    return out


def msc_agreement(cx: Complex, f, g) -> dict:
    """Counts behind the critical / separatrix recall and precision of Section 5.1, from the two
    complexes: critical cells of f, of g and of both by dimension; separatrices of f and g by
    family (0 descending, 1 ascending) and those of f whose counterpart in g (the separatrix of the
    same saddle through the same first cell) ends at the same extremum, or follows the same cells."""
    mf, mg = msc(cx, f), msc(cx, g)
    out = {"crit_f": [0] * 4, "crit_g": [0] * 4, "crit_common": [0] * 4,
           "sep_f": [0, 0], "sep_g": [0, 0], "sep_same_ends": [0, 0], "sep_same_cells": [0, 0]}
    for d in range(cx.top + 1):
        a, b = set(mf.crit[d].tolist()), set(mg.crit[d].tolist())
        out["crit_f"][d], out["crit_g"][d], out["crit_common"][d] = len(a), len(b), len(a & b)
    for k, fam in enumerate(("desc", "asc")):
        sf = _separatrices(*(getattr(mf, f"{fam}_{x}") for x in ("saddle", "offsets", "cells", "terminal")))
        sg = _separatrices(*(getattr(mg, f"{fam}_{x}") for x in ("saddle", "offsets", "cells", "terminal")))
        out["sep_f"][k], out["sep_g"][k] = len(sf), len(sg)
        for key, (term, seq) in sf.items():
            if key in sg:
                out["sep_same_ends"][k] += sg[key][0] == term
                out["sep_same_cells"][k] += sg[key] == (term, seq)
    return out


def edit_bits(q_max: int) -> int:
    """Bits per code of the edit stream: codes 0..q_max are edit counts, q_max + 1 marks a
    lossless vertex, so the least b with 2^b >= q_max + 2."""
    b = 1
    while 2 ** b < q_max + 2:
        b += 1
    return b


def pack_edits(q, q_max: int) -> np.ndarray:
    """The fixed-bit edit stream of Section 4.7 as uint32 words: vertex k's code (q, or q_max + 1
    where q == 0xFF) in bits [k*b, (k+1)*b), least significant bit first."""
    q = np.asarray(q, dtype=np.uint8).reshape(-1)
    b = edit_bits(q_max)
    codes = np.where(q == 0xFF, q_max + 1, q).astype(np.uint32)
    bits = ((codes[:, None] >> np.arange(b, dtype=np.uint32)[None, :]) & 1).astype(np.uint8).reshape(-1)
    words = (len(bits) + 31) // 32
    bits = np.concatenate([bits, np.zeros(words * 32 - len(bits), np.uint8)])
    return np.packbits(bits, bitorder="little").view("<u4").copy()


def unpack_edits(words, n: int, q_max: int) -> np.ndarray:
    """Inverse of pack_edits: the q of n vertices (0xFF for the lossless code)."""
    b = edit_bits(q_max)
    bits = np.unpackbits(np.asarray(words, dtype="<u4").view(np.uint8), bitorder="little")[:n * b]
    codes = (bits.reshape(n, b).astype(np.uint32) << np.arange(b, dtype=np.uint32)[None, :]).sum(1)
    return np.where(codes == q_max + 1, 0xFF, codes).astype(np.uint8)


def bounds(f, xi: float):
    f = _f32(f)
    lo = np.zeros_like(f)
    hi = np.zeros_like(f)
    lib().oracle_bounds(_p(f, PF), f.size, C.c_float(xi), _p(lo, PF), _p(hi, PF))
    return lo, hi


STATUS = {0: "ok", 1: "not_converged", -1: "invalid", -2: "bound", -3: "nonfinite"}
STAT_KEYS = ["iterations", "c_iterations", "s_iterations", "n_edited", "n_quantized", "n_lossless",
             "residual_violations", "converged", "stalled", "status"]
LOG_KEYS = ["kind", "FP0", "FN0", "FP1", "FN1", "FP2", "FN2", "FP3", "FN3", "TM_desc", "TM_asc",
            "n_req", "changed"]


def correct(cx: Complex, f, g_hat, xi: float, tier: int = 4, q_max: int = 6, max_iters: int = 1 << 40,
            log_cap: int = 100000, saddle_saddle: bool = False) -> dict:
    """The correction (Sections 4.3-4.5); saddle_saddle adds the saddle-saddle connectors of a 3D
    complex to the separatrix step at tier 4 (log word 13 counts their troublemakers)."""
    f = _f32(f)
    g_hat = _f32(g_hat)
    g = np.zeros_like(f)
    q = np.zeros(f.size, dtype=np.uint8)
    stats = np.zeros(10, dtype=np.int64)
    log = np.zeros((max(log_cap, 1), 16), dtype=np.int64)
    rc = lib().oracle_correct(cx.h, _p(f, PF), _p(g_hat, PF), C.c_float(xi), tier, int(saddle_saddle), q_max,
                              max_iters,
                              _p(g, PF), _p(q, P8), _p(stats, P64), _p(log, P64), log_cap)
    st = dict(zip(STAT_KEYS, (int(x) for x in stats)))
    out = {"status": STATUS[rc], "stats": st}
    if rc >= 0:
        idx = np.nonzero(q == 0xFF)[0].astype(np.int64)
        out.update(g=g, q=q, lossless_idx=idx, lossless_val=g[idx].copy(),
                   log=log[:min(st["iterations"], log_cap)].copy())
    return out


def residual(cx: Complex, f, g, tier: int = 4, saddle_saddle: bool = False):
    """Violations of g against f (what the correction loop would fix next): an int64 array of
    (dimension, cell id) rows -- cells whose criticality differs, else at tier >= 3 the first
    differing cell of each checked separatrix branch."""
    f = _f32(f)
    g = _f32(g)
    L = lib()
    z = np.zeros(1, dtype=np.int64)
    ss = int(saddle_saddle)
    n = L.oracle_residual(cx.h, _p(f, PF), _p(g, PF), tier, ss, _p(z, P64), _p(z, P64), 0)
    dims = np.zeros(max(n, 1), dtype=np.int64)
    ids = np.zeros(max(n, 1), dtype=np.int64)
    L.oracle_residual(cx.h, _p(f, PF), _p(g, PF), tier, ss, _p(dims, P64), _p(ids, P64), n)
    return np.stack([dims[:n], ids[:n]], axis=1)


def decode(g_hat, q, lossless_idx, lossless_val, xi: float, q_max: int):
    g_hat = _f32(g_hat)
    q = np.ascontiguousarray(q, dtype=np.uint8).reshape(-1)
    idx = np.ascontiguousarray(lossless_idx, dtype=np.int64)
    val = _f32(lossless_val)
    out = np.zeros_like(g_hat)
    lib().oracle_decode(_p(g_hat, PF), _p(q, P8), g_hat.size, _p(idx, P64), _p(val, PF), idx.size,
                        C.c_float(xi), q_max, _p(out, PF))
    return out
