#!/usr/bin/env python3
"""Throughput of the MSC-preserving correction on one MI355X.

A step is one full correction of one field (setup, gradient of f, separatrices of f, C/S loop
to convergence, outputs) through the C ABI, with f and g_hat resident in HBM.  The default
workload is the 2048x2048 field (256 Gaussians + 4-octave value noise, g_hat = f + U[-xi, xi],
xi = 1e-4 * range, tier 4, q_max 6).

Prints one JSON line: MB/s of fp32 input field (4*N bytes per step / step time), per-step
latency percentiles, the roofline of the dominant kernel (measured with HIP events on the
library's launch stream over the timed steps), and the plain CPU oracle timed on a bounded
crop of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MSC-correction MB/s of fp32 field to convergence; p50/p99 batch latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per work unit.  Planes (cell types) per anchor: 6 (2D), 26 (3D).
def bytes_per_unit(family: str, ndim: int) -> float:
    nb = 6 if ndim == 2 else 26
    return {
        "gradient": 4.0 + nb,     # dense pass: read the field once, write every cell's code byte
        "classify": 2.0 * nb + 4,  # dense pass: read f and g codes, write the violation mask
        "setup": 18.0,            # read f, g_hat; write floor, g, state, request
    }.get(family, 0.0)


def loop_bytes(log, ndim: int) -> float:
    """Algorithmic bytes of the correction loop from its per-iteration work counters: a dirty
    vertex reads its value and writes its cells' codes and the next field's copy (8 + NB); an
    affected anchor reads f and g codes and writes its mask (2 NB + 4); a listed anchor reads its
    list entry and mask (8); a requested vertex reads state, g_hat and floor and writes state and
    value (14); a branch cell touched or examined reads its id and two codes (6)."""
    nb = 6 if ndim == 2 else 26
    L = log.astype("float64")
    return float((L[:, 13] * (8 + nb) + L[:, 14] * (2 * nb + 4) + L[:, 15] * 8 + L[:, 11] * 14 +
                  (L[:, 17] + L[:, 18]) * 6).sum())


def workload(name: str):
    from paper_2409_17346_amd import synth
    if name == "large2d":
        return synth.config_large2d()
    if name == "small2d":
        return synth.config_small2d()
    if name == "atoms3d":
        return synth.config_atoms3d()
    raise SystemExit(f"unknown workload {name}")


def sources_sha256() -> str:
    """Hash of the HIP sources (every kernel is in them)."""
    d = os.path.join(ROOT, "paper_2409_17346_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip")):
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def traffic_from_profiles(kernel_file: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != sources_sha256():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, iterations: int, sample_iters: int):
    """The oracle (single thread, as written) on the same full input, timed over a bounded number
    of iterations and scaled to the whole correction.  The oracle recomputes everything densely in
    every iteration, so its cost is a fixed part (building the complex, f's gradient and
    separatrices, the first detection: the run with max_iters = 0) plus a per-iteration part
    (from a run with max_iters = sample_iters); the estimate is fixed + per_iteration * iterations,
    with iterations the full correction's count (equal on both sides by the parity tests)."""
    import oracle
    nx, ny, nz = w.dims
    cx = oracle.Complex.grid(nx, ny, nz)
    f, g = w.f.reshape(-1), w.g_hat.reshape(-1)
    t0 = time.perf_counter()
    oracle.correct(cx, f, g, w.xi, w.tier, w.q_max, max_iters=0)
    fixed = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = oracle.correct(cx, f, g, w.xi, w.tier, w.q_max, max_iters=sample_iters)
    part = time.perf_counter() - t0
    done = r["stats"]["iterations"]
    per_it = max(part - fixed, 0.0) / max(done, 1)
    est = fixed + per_it * iterations
    return {"value": round(4.0 * w.f.size / est / 1e6, 4), "unit": "MB/s", "cores": 1, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"full {'x'.join(map(str, w.f.shape))} input: setup and first detection {fixed:.1f} s, then "
                      f"{done} iterations in {part - fixed:.1f} s on one host thread; scaled to the correction's "
                      f"{iterations} iterations = {est:.0f} s",
            "seconds_estimated": round(est, 1)}


def bench_batch(args):
    """The batched form: a step is one dmt_correct_batch call over 64 uneven fields (32 2D with
    side log-uniform in [256, 1024], 32 3D with side log-uniform in [64, 160], xi from
    {1e-3, 1e-4} * range, g_hat binned or noisy), with launch shapes from the autotuner.  The same
    fields are also corrected one after another by 64 plain dmt_correct calls on one stream."""
    import numpy as np
    import torch
    from paper_2409_17346_amd import autotune, dmt, synth
    ws = synth.batch_mix(0, 64)
    n_total = sum(w.f.size for w in ws)
    print(f"[bench] batch of {len(ws)} fields, {n_total} vertices", file=sys.stderr, flush=True)
    ctx = dmt.Context(0)
    fields = [(torch.from_numpy(w.f).cuda(), torch.from_numpy(w.g_hat).cuda(), w.xi) for w in ws]
    outs = [(torch.empty_like(f), torch.empty(f.shape, dtype=torch.uint8, device="cuda")) for f, _, _ in fields]
    tuning, table = None, []
    if not args.no_tune:
        tuning, table = autotune.tune_batch(ctx, fields, outs, log=lambda m: print(m, file=sys.stderr, flush=True))
        print(f"[bench] tuned: {tuning}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        res = dmt.dmt_correct_batch(ctx, fields, outputs=outs)
        print(f"[bench] warmup {i}: " + str({s: sum(r.status == s for r in res) for s in set(r.status for r in res)}),
              file=sys.stderr, flush=True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        res = dmt.dmt_correct_batch(ctx, fields, outputs=outs, lossless=False)
        lat.append(time.perf_counter() - ts)
        print(f"[bench] step {i}: {lat[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the plain path on the same fields: 64 dmt_correct calls, one after another, one stream
    seq_out = [(torch.empty_like(f), torch.empty(f.shape, dtype=torch.uint8, device="cuda")) for f, _, _ in fields]
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for (f, gh, xi), (go, qo) in zip(fields, seq_out):
        dmt.dmt_correct(ctx, f, gh, xi, 4, 6, want_edits=False, g_out=go, q_out=qo)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - ts
    same = all(torch.equal(a[0].view(torch.int32), b[0].view(torch.int32)) and torch.equal(a[1], b[1])
               for a, b in zip(outs, seq_out))
    print(f"[bench] 64 sequential calls: {seq_s * 1e3:.1f} ms, outputs identical: {same}", file=sys.stderr,
          flush=True)
    dmt.dmt_profile_enable(ctx, True)
    res = dmt.dmt_correct_batch(ctx, fields, outputs=outs)
    prof = dmt.dmt_profile_read(ctx)
    dmt.dmt_profile_enable(ctx, False)
    lat_sorted = sorted(lat)

    def pct(p):
        k = min(len(lat_sorted) - 1, max(0, int(round(p / 100.0 * (len(lat_sorted) - 1)))))
        return round(lat_sorted[k] * 1e3, 3)

    status = {s: sum(r.status == s for r in res) for s in sorted(set(r.status for r in res))}
    iters = [r.stats["iterations"] for r in res]
    line = {
        "metric": METRIC, "value": round(4.0 * n_total * args.steps / elapsed / 1e6, 3), "unit": "MB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64-mixed-2d256-1024-3d64-160", "fields": len(ws), "vertices": n_total,
                   "tier": 4, "q_max": 6, "status": status, "iterations_max": max(iters),
                   "iterations_median": int(np.median(iters)), "tuning": tuning,
                   "tuning_candidates_timed": len(table)},
        "latency_ms": {"p50": pct(50), "p99": pct(99)},
        "sequential": {"ms": round(seq_s * 1e3, 3), "value": round(4.0 * n_total / seq_s / 1e6, 3), "unit": "MB/s",
                       "outputs_identical": same, "speedup_of_batch": round(seq_s / (elapsed / args.steps), 3)},
        "kernel_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def _arrival_stream(qps: float, n: int, seed: int):
    import numpy as np
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / qps, size=n))


def _run_served(dmt, torch, reqs, arrivals, log_every: int = 50):
    """Continuous batching: requests enter dmt_server as they arrive.  Returns latencies (s),
    statuses and the stream's wall time (first arrival to last completion)."""
    srv = dmt.Server(0, hbm_budget_bytes=96 << 30, max_jobs=64)
    outs = {}
    t0 = time.perf_counter()
    nxt, live, lat, status, t_last = 0, {}, [None] * len(reqs), {}, t0
    while nxt < len(reqs) or live:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            f, g, xi = reqs[nxt][:3]
            live[srv.submit(f, g, xi)] = nxt
            nxt += 1
        for t in list(live):
            res = srv.poll(t, lossless=False)
            if res is not None:
                j = live.pop(t)
                t_last = time.perf_counter()
                lat[j] = t_last - t0 - arrivals[j]
                outs[j] = (res.g, res.q)
                status[res.status] = status.get(res.status, 0) + 1
                done = sum(x is not None for x in lat)
                if done % log_every == 0:
                    print(f"[bench] served: {done} done", file=sys.stderr, flush=True)
        if not live and nxt < len(reqs):
            time.sleep(max(0.0, min(0.002, arrivals[nxt] - (time.perf_counter() - t0))))
        else:
            time.sleep(0.0002)
    srv.close()
    return lat, status, t_last - t0, outs


def _run_fifo(dmt, torch, ctx, reqs, arrivals, log_every: int = 50):
    """The plain path under the same arrivals: one dmt_correct at a time, in arrival order."""
    t0 = time.perf_counter()
    lat, status, outs = [], {}, {}
    for j, (f, g, xi, _) in enumerate(reqs):
        wait = arrivals[j] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        go, qo = torch.empty_like(f), torch.empty(f.shape, dtype=torch.uint8, device="cuda")
        r = dmt.dmt_correct(ctx, f, g, xi, 4, 6, want_edits=False, g_out=go, q_out=qo)
        lat.append(time.perf_counter() - t0 - arrivals[j])
        outs[j] = (go, qo)
        status[r.status] = status.get(r.status, 0) + 1
        if (j + 1) % log_every == 0:
            print(f"[bench] fifo: {j + 1} done", file=sys.stderr, flush=True)
    return lat, status, time.perf_counter() - t0, outs


def bench_served(args):
    """The served form: a Poisson stream of correction requests (synth.served_job: 5% 384^3
    lognormal fields, the rest like the batch mix, xi = 1e-4 * range).  The plain path's capacity
    is measured first (every request through dmt_correct back to back); the stream then arrives at
    0.5x and 0.8x that rate, once into dmt_server (continuous batching) and once through the plain
    path one request at a time in arrival order (FIFO).  Reports MB/s of fields completed and
    p50/p99 latency (arrival to completion) of each, and checks that every request's outputs are
    the same in both."""
    import numpy as np
    import torch
    from paper_2409_17346_amd import dmt, synth
    n = args.requests
    t0 = time.perf_counter()
    reqs = []
    for j in range(n):
        w = synth.served_job(j)
        reqs.append((torch.from_numpy(w.f).cuda(), torch.from_numpy(w.g_hat).cuda(), w.xi, w.f.size))
        if (j + 1) % 50 == 0:
            print(f"[bench] generated {j + 1} requests ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    n_big = sum(1 for r in reqs if r[3] == 384 ** 3)
    total_bytes = 4.0 * sum(r[3] for r in reqs)
    ctx = dmt.Context(0)
    # warm both paths on a few requests (kernels loaded, buffers grown)
    for f, g, xi, _ in reqs[:max(1, args.warmup)]:
        dmt.dmt_correct(ctx, f, g, xi, 4, 6, want_edits=False)
    cap_lat, _, cap_s, _ = _run_fifo(dmt, torch, ctx, reqs, np.zeros(n))
    capacity = n / cap_s
    print(f"[bench] plain capacity {capacity:.2f} req/s ({cap_s:.1f} s for {n} requests)", file=sys.stderr,
          flush=True)
    runs = {}
    for load in (0.5, 0.8):
        qps = load * capacity
        arr = _arrival_stream(qps, n, 6000)
        s_lat, s_st, s_wall, s_out = _run_served(dmt, torch, reqs, arr)
        f_lat, f_st, f_wall, f_out = _run_fifo(dmt, torch, ctx, reqs, arr)
        same = all(torch.equal(s_out[j][0].view(torch.int32), f_out[j][0].view(torch.int32)) and
                   torch.equal(s_out[j][1], f_out[j][1]) for j in range(n))

        def summary(lat, st, wall):
            ms = np.array(lat) * 1e3
            return {"value": round(total_bytes / wall / 1e6, 3), "unit": "MB/s", "wall_s": round(wall, 3),
                    "p50_ms": round(float(np.percentile(ms, 50)), 3), "p99_ms": round(float(np.percentile(ms, 99)), 3),
                    "status": st}

        runs[f"load{load}"] = {"qps": round(qps, 3), "served": summary(s_lat, s_st, s_wall),
                               "fifo": summary(f_lat, f_st, f_wall), "outputs_identical": same}
        print(f"[bench] load {load}: {json.dumps(runs[f'load{load}'])}", file=sys.stderr, flush=True)
    head = runs["load0.8"]["served"]
    line = {
        "metric": METRIC, "value": head["value"], "unit": "MB/s", "n_gpus": 1, "steps": n,
        "warmup": args.warmup, "ms_per_step": round(head["wall_s"] / n * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served-poisson-{n}req-5pct-384cubed", "requests": n, "big_requests": n_big,
                   "tier": 4, "q_max": 6, "plain_capacity_rps": round(capacity, 3),
                   "plain_back_to_back": {"value": round(total_bytes / cap_s / 1e6, 3), "unit": "MB/s",
                                          "wall_s": round(cap_s, 3)}},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]},
        "loads": runs,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def _edit_sizes(ctx, dmt, torch, r, w, q_max: int) -> dict:
    """Storage of a correction's edits (Section 4.7, Table 5): the fixed-bit stream plus lossless
    values after DEFLATE (standing in for ZSTD), beside the same edits as floating key-value pairs
    (vertex index int32, delta = g' - g_hat fp32, DEFLATE), and, for 2*xi-bin g_hat, the overall
    compression ratio with the bin indices under DEFLATE as the base compressor's output."""
    import zlib

    import numpy as np
    stream, val = dmt.dmt_pack_edits(ctx, r.q, r.g, q_max)
    blob = dmt.compress_edits(stream, val)
    q = r.q.cpu().numpy().reshape(-1)
    idx = np.nonzero(q)[0]
    delta = (r.g.cpu().numpy().reshape(-1)[idx].astype(np.float64) - w.g_hat.reshape(-1)[idx]).astype(np.float32)
    floating = zlib.compress(idx.astype(np.int32).tobytes() + delta.tobytes(), 9)
    out = {"edit_bytes": len(blob), "stream_bits": int(stream.numel() * 32), "lossless_values": int(val.numel()),
           "floating_edit_bytes": len(floating), "edit_ratio": round(len(idx) / q.size, 6)}
    if w.meta.get("ghat") == "bin":
        codes = np.rint(w.f.astype(np.float64) / (2.0 * w.xi)).astype(np.int32)
        base = len(zlib.compress(codes.tobytes(), 9))
        raw = 4 * q.size
        out.update(base_bytes=base, cr=round(raw / base, 3), ocr=round(raw / (base + len(blob)), 3),
                   ocr_floating=round(raw / (base + len(floating)), 3))
    return out


def _timed_correct(ctx, dmt, torch, w, tier: int, q_max: int, reps: int = 3):
    f = torch.from_numpy(w.f).cuda()
    gh = torch.from_numpy(w.g_hat).cuda()
    best, r = float("inf"), None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dmt.dmt_correct(ctx, f, gh, w.xi, tier, q_max)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best, r, f


def bench_sweep(args):
    """Sweeps on synthetic stand-ins of the paper's studies (one JSON line, entries under "sweep"):
    qmax    - Section 5.5 / Figure 10: q_max 2..7 at relative bounds 1e-5..1e-2 on a 150 x 450 2D
              field (Heated Flow's shape): time, iterations, edit storage and OCR;
    tiers   - Section 5.3 / Figure 11: tiers 1-4 at relative bounds 1e-4..1e-2 on a 361 x 576 2D
              field (IVT's shape): time, iterations, edit storage, and the MSC agreement
              (critical / separatrix recall and precision, Section 5.1) each tier reaches;
    extreme - Section 5.9 / Figure 14: i.i.d. noise in [0, xi) with the absolute bound xi = 1e-4, so
              g_hat is flat, at sides 64..2048: time, iterations and how much of the field is edited."""
    import numpy as np
    import torch
    from paper_2409_17346_amd import dmt, synth
    ctx = dmt.Context(0)
    rows, total_bytes, total_s = [], 0.0, 0.0
    kind = args.workload.split("-", 1)[1]
    if kind == "qmax":
        cases = [(synth.flow2d(150, 450, 3, rel), 4, qm) for rel in (1e-5, 1e-4, 1e-3, 1e-2) for qm in range(2, 8)]
    elif kind == "tiers":
        cases = [(synth.flow2d(361, 576, 4, rel), t, 6) for rel in (1e-4, 1e-3, 1e-2) for t in (1, 2, 3, 4)]
    else:
        cases = [(synth.extreme_noise2d(side, 1), 4, 6) for side in (64, 128, 256, 512, 1024, 2048)]
    for w, tier, q_max in cases:
        sec, r, f = _timed_correct(ctx, dmt, torch, w, tier, q_max)
        row = {"field": w.name, "tier": tier, "q_max": q_max, "ms": round(sec * 1e3, 3),
               "mb_per_s": round(4.0 * w.f.size / sec / 1e6, 3), "status": r.status,
               "iterations": r.stats["iterations"], "c_iterations": r.stats["c_iterations"],
               "s_iterations": r.stats["s_iterations"], "n_edited": r.stats["n_edited"],
               "n_lossless": r.stats["n_lossless"]}
        row.update(_edit_sizes(ctx, dmt, torch, r, w, q_max))
        if kind == "tiers":
            a = dmt.dmt_compare_msc(ctx, f, r.g)
            row.update({k: round(v, 6) for k, v in a.items() if isinstance(v, float)})
        if kind == "extreme":
            q = r.q.cpu().numpy()
            row["fraction_at_q_max"] = round(float((q == q_max).mean()), 6)
            row["fraction_edited"] = round(float((q != 0).mean()), 6)
        rows.append(row)
        total_bytes += 4.0 * w.f.size
        total_s += sec
        print(f"[bench] {json.dumps(row)}", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": round(total_bytes / total_s / 1e6, 3), "unit": "MB/s", "n_gpus": 1,
        "steps": len(rows), "warmup": 0, "ms_per_step": round(total_s / len(rows) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "runs": len(rows), "timing": "best of 3 per run"},
        "sweep": rows,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large2d", choices=["large2d", "small2d", "atoms3d", "batch64", "served", "sweep-qmax",
                             "sweep-tiers", "sweep-extreme"])
    ap.add_argument("--requests", type=int, default=200, help="served: requests in the stream")
    ap.add_argument("--cpu-sample-iters", type=int, default=40,
                    help="iterations of the oracle timed on the full input for the CPU baseline")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the 128x128 and 256^3 configurations after the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="batch64: keep the default launch shapes")
    ap.add_argument("--flags", type=int, default=0, help="dmt_options.flags (1 dense loop, 2 one launch per phase)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB once (untimed): the reference kernel that scales "
                         "profiler byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the correction of one field runs on one "
              f"MI355X and this build has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_17346_amd import dmt

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload.startswith("sweep-"):
        return bench_sweep(args)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)   # an elementwise kernel: reads and writes copy_probe_mib MiB
        torch.cuda.synchronize()
        del src, dst
    w = workload(args.workload)
    ctx = dmt.Context(0)
    line = bench_single(ctx, dmt, torch, w, args.steps, args.warmup, args.flags, full=True)
    if not args.no_extra_configs and args.workload == "large2d" and args.flags == 0:
        # the other single-field configurations, timed the same way (kernel roofline of the headline only)
        extra = {}
        for name, steps in (("small2d", 20), ("atoms3d", 2)):
            wx = workload(name)
            lx = bench_single(ctx, dmt, torch, wx, steps, 1, 0, full=False)
            extra[wx.name] = {"value": lx["value"], "unit": "MB/s", "ms_per_step": lx["ms_per_step"],
                              "steps": steps, "latency_ms": lx["latency_ms"], **lx["config"]}
        line["other_configs"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, line["config"]["iterations"], args.cpu_sample_iters)
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_single(ctx, dmt, torch, w, steps: int, warmup: int, flags: int, full: bool) -> dict:
    """Times `steps` corrections of one field (after `warmup` untimed ones); with full, also the
    kernel rooflines from one more profiled correction."""
    print(f"[bench] workload {w.name} shape {w.f.shape} xi {w.xi:.6g}", file=sys.stderr, flush=True)
    f = torch.from_numpy(w.f).cuda()
    gh = torch.from_numpy(w.g_hat).cuda()
    g_out = torch.empty_like(f)
    q_out = torch.empty(f.shape, dtype=torch.uint8, device="cuda")
    n = f.numel()

    for i in range(warmup):
        r = dmt.dmt_correct(ctx, f, gh, w.xi, w.tier, w.q_max, want_edits=False, g_out=g_out, q_out=q_out,
                            flags=flags)
        print(f"[bench] warmup {i}: {r.status} {r.stats}", file=sys.stderr, flush=True)

    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        r = dmt.dmt_correct(ctx, f, gh, w.xi, w.tier, w.q_max, want_edits=False, g_out=g_out, q_out=q_out,
                            flags=flags)
        lat.append(time.perf_counter() - ts)
        print(f"[bench] step {i}: {lat[-1] * 1e3:.1f} ms {r.status} iterations={r.stats['iterations']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = 4.0 * n * steps / elapsed / 1e6
    lat_sorted = sorted(lat)

    def pct(p):
        k = min(len(lat_sorted) - 1, max(0, int(round(p / 100.0 * (len(lat_sorted) - 1)))))
        return round(lat_sorted[k] * 1e3, 3)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "MB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(elapsed / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(w.dims), "tier": w.tier, "q_max": w.q_max,
                   "rel_error_bound": w.meta.get("rel"), "status": r.status, "iterations": r.stats["iterations"],
                   "c_iterations": r.stats["c_iterations"], "s_iterations": r.stats["s_iterations"],
                   "residual_violations": r.stats["residual_violations"]},
        "latency_ms": {"p50": pct(50), "p99": pct(99)},
    }
    if not full:
        return line
    # kernel timing: one more (untimed) step with HIP events around the library's launches, which
    # also returns the per-iteration work counters
    dmt.dmt_profile_enable(ctx, True)
    rp = dmt.dmt_correct(ctx, f, gh, w.xi, w.tier, w.q_max, want_edits=True, g_out=g_out, q_out=q_out, flags=flags)
    prof = dmt.dmt_profile_read(ctx)
    dmt.dmt_profile_enable(ctx, False)
    ndim = w.ndim

    def roof(fam, alg_total):
        p = prof[fam]
        avg_ms = p["ms"] / p["launches"]
        alg = alg_total / p["launches"]
        achieved = alg / (avg_ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic_from_profiles(f"{fam}_{w.name}.txt"),
                "launches": p["launches"], "avg_launch_us": round(avg_ms * 1e3, 3), "alg_bytes_per_launch": int(alg)}

    # the dominant kernel is the correction loop (resident workgroup loop plus its grid hand-offs)
    line["roofline"] = roof("loop", loop_bytes(rp.log.numpy(), ndim))
    line["roofline_dense_gradient"] = roof("gradient", bytes_per_unit("gradient", ndim) * prof["gradient"]["units"])
    line["roofline_dense_classify"] = roof("classify", bytes_per_unit("classify", ndim) * prof["classify"]["units"])
    line["kernel_ms"] = {k: round(v["ms"], 3) for k, v in prof.items()}
    return line


if __name__ == "__main__":
    main()
