"""Autotuner of the correction loop's launch shapes (dmt_tuning in include/dmt.h).

The knobs are the resident loop's workgroup size per dimension, the hand-off limit above which an
iteration runs as full-grid launches, and how many iterations each hand-off runs.  They change
speed only, so tuning is a timing search: coordinate descent from the current setting, one knob
at a time over a short candidate list, keeping the fastest value.  Every candidate's outputs are
compared bit for bit with the first run's, so a tuning that changed a result would stop the search
with an error instead of being chosen.
"""
from __future__ import annotations

import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from . import dmt

# (knob, index) -> candidate values; index 0/1 = 2D/3D jobs (grid_iterations: single/batch);
# single calls tune handoff_anchors, batches batch_handoff_anchors
CANDIDATES: Dict[Tuple[str, int], Sequence[int]] = {
    ("loop_threads", 0): (1024, 512),
    ("loop_threads", 1): (512, 256),
    ("handoff_anchors", 0): (2048, 8192, 32768),
    ("handoff_anchors", 1): (1024, 8192, 32768),
    ("grid_iterations", 0): (2, 4, 16),
    ("grid_iterations", 1): (4, 16, 64, 256),
    ("batch_handoff_anchors", 0): (2048, 8192, 32768),
    ("batch_handoff_anchors", 1): (2048, 8192, 32768),
}


def _knobs_for(dims: Sequence[int], batch: bool) -> List[Tuple[str, int]]:
    """The knobs a workload exercises: per-dimension knobs of the dimensions it holds."""
    out = []
    for d in sorted(set(dims)):
        i = d - 2
        out += [("loop_threads", i), ("batch_handoff_anchors" if batch else "handoff_anchors", i)]
    out.append(("grid_iterations", 1 if batch else 0))
    return out


def _timed(run: Callable[[], list], repeats: int) -> Tuple[float, list]:
    best, outs = float("inf"), None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = run()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, outs


def _same(a: list, b: list) -> bool:
    return all(torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y) for x, y in zip(a, b))


def tune(ctx: dmt.Context, run: Callable[[], list], dims: Sequence[int], batch: bool, repeats: int = 1,
         log: Optional[Callable[[str], None]] = None) -> Tuple[Dict[str, list], List[dict]]:
    """Tunes ctx for the workload `run` (a callable that runs it once on ctx and returns its output
    tensors), whose jobs have the dimensions `dims`.  Leaves the best setting on ctx and returns it
    with the table of every timing taken."""
    current = dmt.dmt_get_tuning(ctx)
    base_t, base_out = _timed(run, repeats)
    table = [{"tuning": current, "seconds": round(base_t, 4)}]
    best_t = base_t
    for knob, i in _knobs_for(dims, batch):
        for v in CANDIDATES[(knob, i)]:
            if current[knob][i] == v:
                continue
            trial = {k: list(x) for k, x in current.items()}
            trial[knob][i] = v
            dmt.dmt_set_tuning(ctx, trial)
            t, out = _timed(run, repeats)
            if not _same(out, base_out):
                dmt.dmt_set_tuning(ctx, current)
                raise RuntimeError(f"tuning {trial} changed a result")
            table.append({"tuning": trial, "seconds": round(t, 4)})
            if log:
                log(f"[tune] {knob}[{i}]={v}: {t * 1e3:.1f} ms (best {best_t * 1e3:.1f} ms)")
            if t < best_t:
                best_t, current = t, trial
        dmt.dmt_set_tuning(ctx, current)
    return current, table


def tune_single(ctx: dmt.Context, f: torch.Tensor, g_hat: torch.Tensor, xi: float, tier: int = 4, q_max: int = 6,
                repeats: int = 2, log=None):
    """Tunes ctx for repeated dmt_correct calls on one field."""
    g_out = torch.empty_like(f)
    q_out = torch.empty(f.shape, dtype=torch.uint8, device=f.device)

    def run():
        dmt.dmt_correct(ctx, f, g_hat, xi, tier, q_max, want_edits=False, g_out=g_out, q_out=q_out)
        return [g_out.clone(), q_out.clone()]

    return tune(ctx, run, [f.dim()], batch=False, repeats=repeats, log=log)


def tune_batch(ctx: dmt.Context, fields, outputs, tier: int = 4, q_max: int = 6, repeats: int = 1, log=None):
    """Tunes ctx for dmt_correct_batch over fields [(f, g_hat, xi)] with preallocated outputs."""

    def run():
        dmt.dmt_correct_batch(ctx, fields, tier=tier, q_max=q_max, outputs=outputs, lossless=False)
        return [t.clone() for g, q in outputs for t in (g, q)]

    return tune(ctx, run, [f.dim() for f, _, _ in fields], batch=True, repeats=repeats, log=log)
