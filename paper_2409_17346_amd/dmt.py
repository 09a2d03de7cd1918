"""Thin Python binding of the C ABI in include/dmt.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Fields are torch tensors on the
GPU, shaped (ny, nx) for 2D or (nz, ny, nx) for 3D (x fastest, fp32, contiguous); the current
torch stream of the tensor's device is passed as the HIP stream.  PyTorch provides device
memory and streams only: all computation happens in the HIP library ``libdmt.so``.  There is
no CPU fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass
from typing import Dict, Optional, Tuple

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libdmt.so")

DMT_OK = 0
DMT_W_NOT_CONVERGED = 1
DMT_W_PENDING = 2
DMT_E_INVALID = -1
DMT_E_NOMEM = -4
DMT_NOALLOC_SCRATCH_BYTES = 134217728   # include/dmt.h: scratch of dmt_correct_noalloc per GPU
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "pending", -1: "invalid", -2: "bound", -3: "nonfinite",
                -4: "nomem", -5: "hip"}
LOG_WORDS = 21
LOG_KEYS = ["kind", "FP0", "FN0", "FP1", "FN1", "FP2", "FN2", "FP3", "FN3", "TM_desc", "TM_asc", "n_req",
            "changed", "dirty_vertices", "affected_anchors", "listed_anchors", "branches_settled",
            "branch_cells_examined", "branch_cells_touched", "ticks"]

MSC_ITEMS = {
    "crit0": 0, "crit1": 1, "crit2": 2, "crit3": 3,
    "desc_saddle": 10, "desc_offsets": 11, "desc_cells": 12, "desc_terminal": 13,
    "asc_saddle": 20, "asc_offsets": 21, "asc_cells": 22, "asc_terminal": 23,
    "min_label": 30, "max_label": 31,
}

# Names of every entry point declared in include/dmt.h.
ABI_SYMBOLS = [
    "dmt_context_create", "dmt_context_destroy", "dmt_last_error", "dmt_cell_id_space",
    "dmt_xi_from_relative", "dmt_bounds", "dmt_gradient_pairs", "dmt_extract_msc", "dmt_msc_copy",
    "dmt_correct", "dmt_correct_batch", "dmt_lossless_edits", "dmt_iteration_log", "dmt_apply_edits",
    "dmt_profile_enable", "dmt_profile_read", "dmt_workspace_bytes", "dmt_server_create", "dmt_server_destroy",
    "dmt_server_submit", "dmt_server_poll", "dmt_server_info", "dmt_lossless_list", "dmt_correct_noalloc",
    "dmt_set_tuning", "dmt_get_tuning", "dmt_compare_msc", "dmt_edit_bits", "dmt_pack_edits", "dmt_unpack_edits",
]

PROF_KERNELS = {"gradient": 0, "classify": 1, "apply": 2, "sstep": 3, "setup": 4, "msc": 5, "loop": 6,
                "loop.sapply": 7, "loop.grad": 8, "loop.vr": 9}


class DmtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class dmt_grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64)]


class dmt_options(C.Structure):
    _fields_ = [("tier", C.c_int32), ("q_max", C.c_int32), ("max_iters", C.c_int64), ("flags", C.c_uint32)]


class dmt_stats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("c_iterations", C.c_int64), ("s_iterations", C.c_int64),
                ("n_edited", C.c_int64), ("n_quantized", C.c_int64), ("n_lossless", C.c_int64),
                ("residual_violations", C.c_int64), ("converged", C.c_int32), ("stalled", C.c_int32)]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class dmt_tuning(C.Structure):
    _fields_ = [("loop_threads", C.c_int32 * 2), ("handoff_anchors", C.c_int32 * 2),
                ("grid_iterations", C.c_int32 * 2), ("batch_handoff_anchors", C.c_int32 * 2)]

    def as_dict(self) -> Dict[str, list]:
        return {k: list(getattr(self, k)) for k, _ in self._fields_}


class dmt_msc_agreement(C.Structure):
    _fields_ = [("crit_f", C.c_int64 * 4), ("crit_g", C.c_int64 * 4), ("crit_common", C.c_int64 * 4),
                ("sep_f", C.c_int64 * 2), ("sep_g", C.c_int64 * 2), ("sep_same_ends", C.c_int64 * 2),
                ("sep_same_cells", C.c_int64 * 2)]


class dmt_job(C.Structure):
    _fields_ = [("grid", dmt_grid), ("f", C.c_void_p), ("g_hat", C.c_void_p), ("xi", C.c_float),
                ("opts", dmt_options), ("g_out", C.c_void_p), ("q_out", C.c_void_p), ("status", C.c_int),
                ("stats", dmt_stats)]


_lib = None
VP = C.c_void_p
P64 = C.POINTER(C.c_int64)


def load_library(path: str = SO):
    """Loads libdmt.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with `python -m paper_2409_17346_amd.build`")
    L = C.CDLL(path)
    L.dmt_context_create.argtypes = [C.POINTER(VP), C.c_int]
    L.dmt_context_destroy.argtypes = [VP]
    L.dmt_last_error.restype = C.c_char_p
    L.dmt_last_error.argtypes = [VP]
    L.dmt_cell_id_space.argtypes = [C.POINTER(dmt_grid), P64]
    L.dmt_xi_from_relative.argtypes = [VP, C.POINTER(dmt_grid), VP, C.c_double, C.POINTER(C.c_float), VP]
    L.dmt_bounds.argtypes = [VP, VP, C.c_int64, C.c_float, VP, VP, VP]
    L.dmt_gradient_pairs.argtypes = [VP, C.POINTER(dmt_grid), VP, VP, VP, VP]
    L.dmt_extract_msc.argtypes = [VP, C.POINTER(dmt_grid), VP, P64, VP]
    L.dmt_msc_copy.argtypes = [VP, C.c_int, VP, C.c_int64, VP]
    L.dmt_correct.argtypes = [VP, C.POINTER(dmt_grid), VP, VP, C.c_float, C.POINTER(dmt_options), VP, VP,
                              C.POINTER(dmt_stats), VP]
    L.dmt_correct_batch.argtypes = [VP, C.c_int32, C.POINTER(dmt_job), VP]
    L.dmt_lossless_edits.argtypes = [VP, VP, VP, C.c_int64, P64, VP]
    L.dmt_iteration_log.argtypes = [VP, P64, C.c_int64, P64]
    L.dmt_apply_edits.argtypes = [VP, VP, VP, C.c_int64, VP, VP, C.c_int64, C.c_float, C.c_int32, VP, VP]
    L.dmt_profile_enable.argtypes = [VP, C.c_int]
    L.dmt_profile_read.argtypes = [VP, C.c_int, P64, C.POINTER(C.c_double), P64]
    L.dmt_workspace_bytes.argtypes = [C.POINTER(dmt_grid), C.POINTER(dmt_options)]
    L.dmt_server_create.argtypes = [C.POINTER(VP), C.c_int, C.c_int64, C.c_int32]
    L.dmt_server_destroy.argtypes = [VP]
    L.dmt_server_submit.argtypes = [VP, C.POINTER(dmt_job), P64]
    L.dmt_server_poll.argtypes = [VP, C.c_int64, C.c_int32, C.POINTER(dmt_job)]
    P32 = C.POINTER(C.c_int32)
    L.dmt_server_info.argtypes = [VP, P64, P64, P32, P32, P32]
    L.dmt_lossless_list.argtypes = [VP, VP, VP, C.c_int64, VP, VP, C.c_int64, P64, VP]
    L.dmt_compare_msc.argtypes = [VP, C.POINTER(dmt_grid), VP, VP, C.POINTER(dmt_msc_agreement), VP]
    L.dmt_edit_bits.argtypes = [C.c_int32]
    L.dmt_edit_bits.restype = C.c_int32
    L.dmt_pack_edits.argtypes = [VP, VP, VP, C.c_int64, C.c_int32, VP, C.c_int64, VP, C.c_int64, P64, VP]
    L.dmt_unpack_edits.argtypes = [VP, VP, C.c_int64, C.c_int64, C.c_int32, VP, VP, C.c_int64, C.c_float, VP, VP,
                                   VP]
    L.dmt_set_tuning.argtypes = [VP, C.POINTER(dmt_tuning)]
    L.dmt_get_tuning.argtypes = [VP, C.POINTER(dmt_tuning)]
    L.dmt_correct_noalloc.argtypes = [VP, C.POINTER(dmt_grid), VP, VP, C.c_float, C.POINTER(dmt_options), VP, VP,
                                      VP, VP, C.c_int64, P64, C.POINTER(dmt_stats), VP]
    for name in ABI_SYMBOLS:
        if name != "dmt_last_error":
            getattr(L, name).restype = C.c_int
    L.dmt_workspace_bytes.restype = C.c_int64
    L.dmt_edit_bits.restype = C.c_int32
    _lib = L
    return L


def grid_of(t: torch.Tensor) -> dmt_grid:
    if t.dim() == 2:
        return dmt_grid(2, t.shape[1], t.shape[0], 1)
    if t.dim() == 3:
        return dmt_grid(3, t.shape[2], t.shape[1], t.shape[0])
    raise ValueError("fields must be 2D (ny, nx) or 3D (nz, ny, nx)")


def _dev(t: torch.Tensor, dtype=torch.float32) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor")
    return t


def _stream(t: torch.Tensor):
    return VP(torch.cuda.current_stream(t.device).cuda_stream)


# Contexts and servers still open when the interpreter exits are closed by an atexit hook, which
# runs before the HIP runtime's own teardown; a destructor left to interpreter finalization could
# otherwise free device memory after the runtime is gone.
_live = weakref.WeakSet()


def _close_all():
    for o in sorted(list(_live), key=lambda o: not isinstance(o, Server)):   # servers first
        try:
            o.close()
        except Exception:
            pass


atexit.register(_close_all)


class Context:
    """Owns a dmt_context (device scratch + results of the last extraction / correction)."""

    def __init__(self, device: int = 0):
        self.L = load_library()
        self.device = device
        h = VP()
        st = self.L.dmt_context_create(C.byref(h), device)
        if st != DMT_OK:
            raise DmtError(st, "dmt_context_create failed")
        self.h = h
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.L.dmt_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st: int, allow=(DMT_OK,)):
        if st not in allow:
            raise DmtError(st, self.L.dmt_last_error(self.h).decode())
        return st


def dmt_context_create(device: int = 0) -> Context:
    return Context(device)


def dmt_cell_id_space(shape) -> Tuple[int, int, int, int]:
    L = load_library()
    g = dmt_grid(2, shape[1], shape[0], 1) if len(shape) == 2 else dmt_grid(3, shape[2], shape[1], shape[0])
    out = (C.c_int64 * 4)()
    st = L.dmt_cell_id_space(C.byref(g), out)
    if st != DMT_OK:
        raise DmtError(st, "invalid grid")
    return tuple(int(x) for x in out)


def dmt_xi_from_relative(ctx: Context, f: torch.Tensor, rel: float) -> float:
    _dev(f)
    xi = C.c_float()
    g = grid_of(f)
    ctx.check(ctx.L.dmt_xi_from_relative(ctx.h, C.byref(g), VP(f.data_ptr()), rel, C.byref(xi), _stream(f)))
    return float(xi.value)


def dmt_bounds(ctx: Context, f: torch.Tensor, xi: float):
    _dev(f)
    lo = torch.empty_like(f)
    hi = torch.empty_like(f)
    ctx.check(ctx.L.dmt_bounds(ctx.h, VP(f.data_ptr()), f.numel(), xi, VP(lo.data_ptr()), VP(hi.data_ptr()),
                               _stream(f)))
    return lo, hi


def dmt_gradient_pairs(ctx: Context, field: torch.Tensor):
    """Returns (up, down) int64 tensors over the concatenated per-dimension cell id spaces."""
    _dev(field)
    counts = dmt_cell_id_space(tuple(field.shape))
    total = sum(counts)
    up = torch.empty(total, dtype=torch.int64, device=field.device)
    down = torch.empty(total, dtype=torch.int64, device=field.device)
    g = grid_of(field)
    ctx.check(ctx.L.dmt_gradient_pairs(ctx.h, C.byref(g), VP(field.data_ptr()), VP(up.data_ptr()),
                                       VP(down.data_ptr()), _stream(field)))
    return up, down, counts


def dmt_extract_msc(ctx: Context, field: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Critical cells, separatrix branches and manifold labels of field, as int64 GPU tensors."""
    _dev(field)
    counts = (C.c_int64 * 32)()
    g = grid_of(field)
    ctx.check(ctx.L.dmt_extract_msc(ctx.h, C.byref(g), VP(field.data_ptr()), counts, _stream(field)))
    out = {}
    for name, item in MSC_ITEMS.items():
        n = int(counts[item])
        t = torch.empty(max(n, 0), dtype=torch.int64, device=field.device)
        if n > 0:
            ctx.check(ctx.L.dmt_msc_copy(ctx.h, item, VP(t.data_ptr()), n, _stream(field)))
        out[name] = t
    return out


@dataclass
class Result:
    status: str
    g: torch.Tensor
    q: torch.Tensor
    stats: Dict[str, int]
    lossless_idx: torch.Tensor
    lossless_val: torch.Tensor
    log: torch.Tensor


DMT_F_DENSE = 1
DMT_F_PHASES = 2
DMT_F_SADDLE_SADDLE = 4


def dmt_correct(ctx: Context, f: torch.Tensor, g_hat: torch.Tensor, xi: float, tier: int = 4, q_max: int = 6,
                max_iters: int = -1, want_edits: bool = True, g_out: torch.Tensor | None = None,
                q_out: torch.Tensor | None = None, flags: int = 0) -> Result:
    _dev(f)
    _dev(g_hat)
    if f.shape != g_hat.shape:
        raise ValueError("f and g_hat differ in shape")
    g_out = torch.empty_like(f) if g_out is None else g_out
    q_out = torch.empty(f.shape, dtype=torch.uint8, device=f.device) if q_out is None else q_out
    st = dmt_stats()
    opts = dmt_options(tier, q_max, max_iters, flags)
    g = grid_of(f)
    rc = ctx.check(ctx.L.dmt_correct(ctx.h, C.byref(g), VP(f.data_ptr()), VP(g_hat.data_ptr()), xi, C.byref(opts),
                                     VP(g_out.data_ptr()), VP(q_out.data_ptr()), C.byref(st), _stream(f)),
                   allow=(DMT_OK, DMT_W_NOT_CONVERGED))
    stats = st.as_dict()
    idx = val = log = None
    if want_edits:
        idx, val = dmt_lossless_edits(ctx, f.device)
        log = dmt_iteration_log(ctx)
    return Result(STATUS_NAMES[rc], g_out, q_out, stats, idx, val, log)


def dmt_compare_msc(ctx: Context, f: torch.Tensor, g: torch.Tensor) -> Dict[str, object]:
    """Agreement of g's MSC with f's (Section 5.1): the raw counts of dmt_msc_agreement plus
    critical and separatrix recall / precision (separatrices: identical cell sequences; the
    *_connectivity variants: same saddle, same first cell, same terminal)."""
    _dev(f)
    _dev(g)
    if f.shape != g.shape:
        raise ValueError("f and g differ in shape")
    a = dmt_msc_agreement()
    ctx.check(ctx.L.dmt_compare_msc(ctx.h, C.byref(grid_of(f)), VP(f.data_ptr()), VP(g.data_ptr()), C.byref(a),
                                    _stream(f)))
    out = {k: list(getattr(a, k)) for k, _ in a._fields_}
    return dict(out, **agreement_rates(out))


def agreement_rates(a: Dict[str, list]) -> Dict[str, float]:
    """Recall (common / f's) and precision (common / g's) from agreement counts; 1.0 for empty sets."""
    def ratio(x, y):
        return 1.0 if y == 0 else x / y
    cc, cf, cg = sum(a["crit_common"]), sum(a["crit_f"]), sum(a["crit_g"])
    sc, se, sf, sg = sum(a["sep_same_cells"]), sum(a["sep_same_ends"]), sum(a["sep_f"]), sum(a["sep_g"])
    return {"critical_recall": ratio(cc, cf), "critical_precision": ratio(cc, cg),
            "separatrix_recall": ratio(sc, sf), "separatrix_precision": ratio(sc, sg),
            "separatrix_recall_connectivity": ratio(se, sf), "separatrix_precision_connectivity": ratio(se, sg)}


def dmt_edit_bits(q_max: int) -> int:
    return int(load_library().dmt_edit_bits(q_max))


def dmt_pack_edits(ctx: Context, q_out: torch.Tensor, g_out: torch.Tensor, q_max: int
                   ) -> Tuple[torch.Tensor, torch.Tensor]:
    """The fixed-bit edit stream (uint32 words) and the lossless values in vertex order."""
    _dev(q_out, torch.uint8)
    _dev(g_out)
    n = q_out.numel()
    b = dmt_edit_bits(q_max)
    if b < 0:
        raise ValueError("q_max must be 0..7")
    words = (n * b + 31) // 32
    stream = torch.empty(max(words, 1), dtype=torch.int32, device=q_out.device)
    cnt = C.c_int64()
    s = _stream(q_out)
    ctx.check(ctx.L.dmt_pack_edits(ctx.h, VP(q_out.data_ptr()), VP(g_out.data_ptr()), n, q_max, VP(stream.data_ptr()),
                                   words, None, 0, C.byref(cnt), s))
    val = torch.empty(cnt.value, dtype=torch.float32, device=q_out.device)
    if cnt.value:
        ctx.check(ctx.L.dmt_pack_edits(ctx.h, VP(q_out.data_ptr()), VP(g_out.data_ptr()), n, q_max,
                                       VP(stream.data_ptr()), words, VP(val.data_ptr()), cnt.value, C.byref(cnt), s))
    return stream[:words], val


def dmt_unpack_edits(ctx: Context, stream: torch.Tensor, lossless_val: torch.Tensor, g_hat: torch.Tensor, xi: float,
                     q_max: int, want_q: bool = True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    """Decoder of dmt_pack_edits: the corrected field (and the edit counts)."""
    _dev(stream, torch.int32)
    _dev(lossless_val)
    _dev(g_hat)
    g = torch.empty_like(g_hat)
    q = torch.empty(g_hat.shape, dtype=torch.uint8, device=g_hat.device) if want_q else None
    ctx.check(ctx.L.dmt_unpack_edits(ctx.h, VP(stream.data_ptr()), stream.numel(), g_hat.numel(), q_max,
                                     VP(g_hat.data_ptr()), VP(lossless_val.data_ptr()), lossless_val.numel(), xi,
                                     VP(g.data_ptr()), VP(q.data_ptr()) if want_q else None, _stream(g_hat)))
    return g, q


def compress_edits(stream: torch.Tensor, lossless_val: torch.Tensor, level: int = 9) -> bytes:
    """The dictionary-coder stage on the host: DEFLATE (zlib) of the edit stream followed by the
    lossless values, standing in for the paper's ZSTD (not available here).  Layout: uint64 stream
    words, uint64 lossless count, the two compressed sections' lengths, then the sections."""
    import struct
    import zlib
    a = zlib.compress(stream.cpu().numpy().tobytes(), level)
    b = zlib.compress(lossless_val.cpu().numpy().tobytes(), level)
    return struct.pack("<QQQQ", stream.numel(), lossless_val.numel(), len(a), len(b)) + a + b


def decompress_edits(blob: bytes, device="cuda") -> Tuple[torch.Tensor, torch.Tensor]:
    import struct
    import zlib

    import numpy as np
    nw, nl, la, lb = struct.unpack_from("<QQQQ", blob, 0)
    a = zlib.decompress(blob[32:32 + la])
    b = zlib.decompress(blob[32 + la:32 + la + lb])
    stream = torch.from_numpy(np.frombuffer(a, dtype=np.int32).copy()).to(device)
    val = torch.from_numpy(np.frombuffer(b, dtype=np.float32).copy()).to(device)
    if stream.numel() != nw or val.numel() != nl:
        raise ValueError("corrupt edit record")
    return stream, val


def dmt_correct_noalloc(ctx: Context, f: torch.Tensor, g_hat: torch.Tensor, xi: float, g_out: torch.Tensor,
                        q_out: torch.Tensor, lossless_idx: torch.Tensor, lossless_val: torch.Tensor, tier: int = 4,
                        q_max: int = 6, max_iters: int = -1, flags: int = 0) -> Result:
    """The allocation-free correction: every output buffer is the caller's (lossless_idx int64 and
    lossless_val float32 of equal length = the list's capacity); the library allocates nothing.
    Returns a Result whose lossless_idx / lossless_val are views of the filled prefixes."""
    for t in (f, g_hat, g_out):
        _dev(t)
    _dev(q_out, torch.uint8)
    _dev(lossless_idx, torch.int64)
    _dev(lossless_val)
    if f.shape != g_hat.shape or f.shape != g_out.shape or f.shape != q_out.shape:
        raise ValueError("f, g_hat, g_out and q_out differ in shape")
    if lossless_idx.numel() != lossless_val.numel():
        raise ValueError("lossless_idx and lossless_val differ in length")
    st = dmt_stats()
    cnt = C.c_int64()
    opts = dmt_options(tier, q_max, max_iters, flags)
    g = grid_of(f)
    rc = ctx.check(ctx.L.dmt_correct_noalloc(ctx.h, C.byref(g), VP(f.data_ptr()), VP(g_hat.data_ptr()), xi,
                                             C.byref(opts), VP(g_out.data_ptr()), VP(q_out.data_ptr()),
                                             VP(lossless_idx.data_ptr()), VP(lossless_val.data_ptr()),
                                             lossless_idx.numel(), C.byref(cnt), C.byref(st), _stream(f)),
                   allow=(DMT_OK, DMT_W_NOT_CONVERGED))
    m = cnt.value
    return Result(STATUS_NAMES[rc], g_out, q_out, st.as_dict(), lossless_idx[:m], lossless_val[:m], None)


def dmt_set_tuning(ctx: Context, tuning: Optional[Dict[str, list]] = None) -> None:
    """Sets the loop's launch shapes ({"loop_threads": [2D, 3D], "handoff_anchors": [2D, 3D],
    "grid_iterations": [single, batch], "batch_handoff_anchors": [2D, 3D]}); keys left out keep
    the context's current values.  None restores the defaults."""
    if tuning is None:
        ctx.check(ctx.L.dmt_set_tuning(ctx.h, None))
        return
    t = dmt_tuning()
    ctx.check(ctx.L.dmt_get_tuning(ctx.h, C.byref(t)))
    for k, v in tuning.items():
        arr = getattr(t, k)
        arr[0], arr[1] = int(v[0]), int(v[1])
    ctx.check(ctx.L.dmt_set_tuning(ctx.h, C.byref(t)))


def dmt_get_tuning(ctx: Context) -> Dict[str, list]:
    t = dmt_tuning()
    ctx.check(ctx.L.dmt_get_tuning(ctx.h, C.byref(t)))
    return t.as_dict()


def dmt_correct_batch(ctx: Context, fields, tier: int = 4, q_max: int = 6, max_iters: int = -1,
                      outputs=None, lossless: bool = True, flags: int = 0):
    """Corrects a list of (f, g_hat, xi) jobs together.  Returns a list of Result (lossless edits
    read by the library from q == 0xFF unless lossless is False; no per-iteration log)."""
    n = len(fields)
    arr = (dmt_job * n)()
    outs = []
    for j, (f, gh, xi) in enumerate(fields):
        _dev(f)
        _dev(gh)
        if outputs is None:
            g_out = torch.empty_like(f)
            q_out = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
        else:
            g_out, q_out = outputs[j]
        outs.append((g_out, q_out))
        arr[j].grid = grid_of(f)
        arr[j].f = f.data_ptr()
        arr[j].g_hat = gh.data_ptr()
        arr[j].xi = xi
        arr[j].opts = dmt_options(tier, q_max, max_iters, flags)
        arr[j].g_out = g_out.data_ptr()
        arr[j].q_out = q_out.data_ptr()
    st = _stream(fields[0][0]) if n else None
    rc = ctx.L.dmt_correct_batch(ctx.h, n, arr, st)
    if rc < 0 and all(arr[j].status >= 0 for j in range(n)):
        raise DmtError(rc, ctx.L.dmt_last_error(ctx.h).decode())
    res = []
    for j in range(n):
        g_out, q_out = outs[j]
        stj = int(arr[j].status)
        idx, val = dmt_lossless_list(ctx, q_out, g_out) if stj >= 0 and lossless else (None, None)
        res.append(Result(STATUS_NAMES.get(stj, str(stj)), g_out, q_out, arr[j].stats.as_dict(), idx, val, None))
    return res


def dmt_lossless_list(ctx: Context, q_out: torch.Tensor, g_out: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """Lossless edits (vertex ids ascending, values) of a finished job, from its q_out and g_out."""
    _dev(q_out, torch.uint8)
    _dev(g_out)
    n = C.c_int64()
    s = _stream(g_out)
    m = g_out.numel()
    ctx.check(ctx.L.dmt_lossless_list(ctx.h, VP(q_out.data_ptr()), VP(g_out.data_ptr()), m, None, None, 0,
                                      C.byref(n), s))
    idx = torch.empty(n.value, dtype=torch.int64, device=g_out.device)
    val = torch.empty(n.value, dtype=torch.float32, device=g_out.device)
    if n.value:
        ctx.check(ctx.L.dmt_lossless_list(ctx.h, VP(q_out.data_ptr()), VP(g_out.data_ptr()), m, VP(idx.data_ptr()),
                                          VP(val.data_ptr()), n.value, C.byref(n), s))
    return idx, val


def dmt_lossless_edits(ctx: Context, device) -> Tuple[torch.Tensor, torch.Tensor]:
    n = C.c_int64()
    s = VP(torch.cuda.current_stream(device).cuda_stream)
    ctx.check(ctx.L.dmt_lossless_edits(ctx.h, None, None, 0, C.byref(n), s))
    idx = torch.empty(n.value, dtype=torch.int64, device=device)
    val = torch.empty(n.value, dtype=torch.float32, device=device)
    if n.value:
        ctx.check(ctx.L.dmt_lossless_edits(ctx.h, VP(idx.data_ptr()), VP(val.data_ptr()), n.value, C.byref(n), s))
    return idx, val


def dmt_iteration_log(ctx: Context) -> torch.Tensor:
    n = C.c_int64()
    ctx.check(ctx.L.dmt_iteration_log(ctx.h, None, 0, C.byref(n)))
    out = torch.zeros((n.value, LOG_WORDS), dtype=torch.int64)
    if n.value:
        ctx.check(ctx.L.dmt_iteration_log(ctx.h, C.cast(out.data_ptr(), P64), n.value, C.byref(n)))
    return out


def dmt_apply_edits(ctx: Context, g_hat: torch.Tensor, q: torch.Tensor, idx: torch.Tensor, val: torch.Tensor,
                    xi: float, q_max: int) -> torch.Tensor:
    _dev(g_hat)
    _dev(q, torch.uint8)
    out = torch.empty_like(g_hat)
    m = idx.numel()
    ctx.check(ctx.L.dmt_apply_edits(ctx.h, VP(g_hat.data_ptr()), VP(q.data_ptr()), g_hat.numel(),
                                    VP(idx.data_ptr()) if m else None, VP(val.data_ptr()) if m else None, m, xi,
                                    q_max, VP(out.data_ptr()), _stream(g_hat)))
    return out


def dmt_profile_enable(ctx: Context, enable: bool = True) -> None:
    ctx.check(ctx.L.dmt_profile_enable(ctx.h, 1 if enable else 0))


def dmt_profile_read(ctx: Context) -> Dict[str, Dict[str, float]]:
    """Per kernel family: launches, total ms (HIP events on the launch stream), work units."""
    out = {}
    for name, k in PROF_KERNELS.items():
        n = C.c_int64()
        ms = C.c_double()
        u = C.c_int64()
        ctx.check(ctx.L.dmt_profile_read(ctx.h, k, C.byref(n), C.byref(ms), C.byref(u)))
        out[name] = {"launches": int(n.value), "ms": float(ms.value), "units": int(u.value)}
    return out


def dmt_workspace_bytes(shape, tier: int = 4, q_max: int = 6) -> int:
    L = load_library()
    g = dmt_grid(2, shape[1], shape[0], 1) if len(shape) == 2 else dmt_grid(3, shape[2], shape[1], shape[0])
    return int(L.dmt_workspace_bytes(C.byref(g), C.byref(dmt_options(tier, q_max, -1, 0))))


class Server:
    """The served form: dmt_server_create / submit / poll / destroy.  Inputs must be complete on
    the device when submitted (the server runs on its own stream); keep the tensors alive until
    the ticket is polled."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 64 << 30, max_jobs: int = 64):
        self.L = load_library()
        h = VP()
        st = self.L.dmt_server_create(C.byref(h), device, hbm_budget_bytes, max_jobs)
        if st != DMT_OK:
            raise DmtError(st, "dmt_server_create failed")
        self.h = h
        _live.add(self)
        self._held = {}
        self._ctx = None   # context for reading lossless lists of finished jobs

    def submit(self, f: torch.Tensor, g_hat: torch.Tensor, xi: float, tier: int = 4, q_max: int = 6,
               max_iters: int = -1, g_out: Optional[torch.Tensor] = None, q_out: Optional[torch.Tensor] = None,
               flags: int = 0) -> int:
        _dev(f)
        _dev(g_hat)
        if g_out is None:
            g_out = torch.empty_like(f)
        if q_out is None:
            q_out = torch.empty(f.shape, dtype=torch.uint8, device=f.device)
        j = dmt_job()
        j.grid = grid_of(f)
        j.f, j.g_hat, j.xi = f.data_ptr(), g_hat.data_ptr(), xi
        j.opts = dmt_options(tier, q_max, max_iters, flags)
        j.g_out, j.q_out = g_out.data_ptr(), q_out.data_ptr()
        torch.cuda.current_stream(f.device).synchronize()   # inputs complete before the server reads them
        t = C.c_int64()
        st = self.L.dmt_server_submit(self.h, C.byref(j), C.byref(t))
        if st != DMT_OK:
            raise DmtError(st, "dmt_server_submit rejected the job")
        self._held[t.value] = (f, g_hat, g_out, q_out)
        return t.value

    def poll(self, ticket: int, wait: bool = False, lossless: bool = True) -> Optional[Result]:
        """Result of a finished ticket (then released), or None while it runs.  With lossless, the
        library also reads the job's lossless edits from its outputs."""
        j = dmt_job()
        st = self.L.dmt_server_poll(self.h, ticket, 1 if wait else 0, C.byref(j))
        if st == DMT_W_PENDING:
            return None
        if st != DMT_OK:
            raise DmtError(st, "unknown ticket")
        f, gh, g_out, q_out = self._held.pop(ticket)
        stj = int(j.status)
        idx = val = None
        if stj >= 0 and lossless:
            if self._ctx is None:
                self._ctx = Context(g_out.device.index or 0)
            idx, val = dmt_lossless_list(self._ctx, q_out, g_out)
        return Result(STATUS_NAMES.get(stj, str(stj)), g_out, q_out, j.stats.as_dict(), idx, val, None)

    def info(self) -> Dict[str, int]:
        """Admission accounting: inflight and held bytes, idle slots, queued jobs."""
        a, b = C.c_int64(), C.c_int64()
        fs, pn, df = C.c_int32(), C.c_int32(), C.c_int32()
        st = self.L.dmt_server_info(self.h, C.byref(a), C.byref(b), C.byref(fs), C.byref(pn), C.byref(df))
        if st != DMT_OK:
            raise DmtError(st, "dmt_server_info failed")
        return {"inflight_bytes": a.value, "held_bytes": b.value, "free_slots": fs.value, "pending": pn.value,
                "distinct_free_slots": df.value}

    def close(self):
        if getattr(self, "h", None):
            self.L.dmt_server_destroy(self.h)
            self.h = None
            self._held.clear()
        if getattr(self, "_ctx", None) is not None:
            self._ctx.close()
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
