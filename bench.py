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


def bench_served(args):
    """The served form: a Poisson stream of correction requests into dmt_server.  Requests draw
    their fields from a pool: 23 fields like the batch mix (2D side 256-1024, 3D side 64-160,
    xi = 1e-4 * range) and one 384^3 lognormal 3D field used by the ~5% large requests.  Reports
    MB/s of fields completed over the stream's wall time and p50/p99 request latency (arrival to
    completion)."""
    import numpy as np
    import torch
    from paper_2409_17346_amd import dmt, synth
    rng = np.random.default_rng(6000)
    big_ids = [j for j in range(args.requests) if np.random.default_rng(5000 + j).uniform() < 0.05]
    small = [synth.served_job(j) for j in range(40) if np.random.default_rng(5000 + j).uniform() >= 0.05][:23]
    big = synth.served_job(big_ids[0]) if big_ids else None
    pool = [(torch.from_numpy(w.f).cuda(), torch.from_numpy(w.g_hat).cuda(), w.xi, w.f.size) for w in small]
    bigt = (torch.from_numpy(big.f).cuda(), torch.from_numpy(big.g_hat).cuda(), big.xi, big.f.size) if big else None
    reqs = [bigt if j in big_ids else pool[int(rng.integers(0, len(pool)))] for j in range(args.requests)]
    arrivals = np.cumsum(rng.exponential(1.0 / args.qps, size=args.requests))
    print(f"[bench] served: {args.requests} requests ({len(big_ids)} of 384^3) at {args.qps} req/s",
          file=sys.stderr, flush=True)
    srv = dmt.Server(0, hbm_budget_bytes=96 << 30, max_jobs=64)
    # warmup: one request of each pool field kind
    for r in reqs[:args.warmup]:
        srv.poll(srv.submit(r[0], r[1], r[2]), wait=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, live, lat, status, done_bytes = 0, {}, [], {}, 0.0
    t_last = t0
    while nxt < len(reqs) or live:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now:
            f, g, xi, n = reqs[nxt]
            live[srv.submit(f, g, xi)] = (arrivals[nxt], n)
            nxt += 1
        for t in list(live):
            res = srv.poll(t)
            if res is not None:
                a, n = live.pop(t)
                t_last = time.perf_counter()
                lat.append(t_last - t0 - a)
                done_bytes += 4.0 * n
                status[res.status] = status.get(res.status, 0) + 1
                if len(lat) % 20 == 0:
                    print(f"[bench] {len(lat)} done, latency p50 {np.percentile(lat, 50):.3f} s", file=sys.stderr,
                          flush=True)
        time.sleep(0.0005)
    elapsed = t_last - t0
    srv.close()
    lat_ms = np.array(lat) * 1e3
    line = {
        "metric": METRIC, "value": round(done_bytes / elapsed / 1e6, 3), "unit": "MB/s", "n_gpus": 1,
        "steps": len(lat), "warmup": args.warmup, "ms_per_step": round(elapsed / len(lat) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"served-poisson-{args.qps}qps-{args.requests}req", "big_requests": len(big_ids),
                   "tier": 4, "q_max": 6, "status": status},
        "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 3),
                       "p99": round(float(np.percentile(lat_ms, 99)), 3)},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large2d", choices=["large2d", "small2d", "atoms3d", "batch64", "served"])
    ap.add_argument("--requests", type=int, default=200, help="served: requests in the stream")
    ap.add_argument("--qps", type=float, default=4.0, help="served: Poisson arrival rate (requests/s)")
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
