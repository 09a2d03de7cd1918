"""Writes tests/golden/full_size.json: the oracle's results on full-size workloads, as hashes.

Run on the CPU (it calls only ``oracle`` and the seeded generators in ``synth``):

    python tests/golden/make_full_size.py [case ...]

Every case regenerates its input from a seeded recipe, runs the plain C oracle to the end and
stores the sha256 of the input arrays and of every output (corrected field bits, quantized edit
counts, lossless edit ids and value bits, the per-iteration log's result words), the statistics,
and how long the oracle took on how many host threads.  The GPU tests regenerate the same inputs,
check their hashes against the stored ones, run the HIP path and compare output hashes.
Cases run in parallel processes; existing entries of other cases are kept.
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "full_size.json")

# name -> (recipe evaluated with synth in scope, tier)
CASES = {
    "2d-2048-gauss256-valuenoise-noise-1e-4": ("synth.config_large2d()", 4),
    "3d-128-lognormal-bin-1e-4": ("synth.lognormal_case(128, 7)", 4),
    "batch0-0-2d-481": ("synth.batch_field(0, 0)", 4),
    "batch0-3-2d-557": ("synth.batch_field(0, 3)", 4),
    "batch0-33-3d-95": ("synth.batch_field(0, 33)", 4),
    "batch0-34-3d-101": ("synth.batch_field(0, 34)", 4),
}


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def output_hashes(g, q, idx, val, log13) -> dict:
    """The hashed form of a correction's outputs (shared by this script and the GPU tests)."""
    return {
        "g_bits": sha(np.asarray(g, np.float32).reshape(-1).view(np.uint32)),
        "q": sha(np.asarray(q, np.uint8).reshape(-1)),
        "lossless_idx": sha(np.asarray(idx, np.int64).reshape(-1)),
        "lossless_val_bits": sha(np.asarray(val, np.float32).reshape(-1).view(np.uint32)),
        "log13": sha(np.asarray(log13, np.int64).reshape(-1, 13)),
    }


def input_hashes(w) -> dict:
    return {"f": sha(w.f.astype(np.float32)), "g_hat": sha(w.g_hat.astype(np.float32)),
            "xi": float(w.xi).hex()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_case(name: str) -> dict:
    import oracle
    from paper_2409_17346_amd import synth
    recipe, tier = CASES[name]
    w = eval(recipe, {"synth": synth})
    nx, ny, nz = w.dims
    t0 = time.perf_counter()
    o = oracle.correct(oracle.Complex.grid(nx, ny, nz), w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, tier, w.q_max)
    sec = time.perf_counter() - t0
    stats = {k: int(v) for k, v in o["stats"].items() if k != "status"}
    return {
        "recipe": recipe, "dims": [nx, ny, nz], "tier": tier, "q_max": w.q_max,
        "input": input_hashes(w), "status": o["status"], "stats": stats,
        "outputs": output_hashes(o["g"], o["q"], o["lossless_idx"], o["lossless_val"], o["log"][:, :13]),
        "n_log": int(o["log"].shape[0]),
        "oracle_seconds": round(sec, 2), "oracle_threads": 1, "cpu": cpu_model(),
    }


def main(names):
    names = names or list(CASES)
    old = json.load(open(OUT)) if os.path.exists(OUT) else {}
    with ProcessPoolExecutor(max_workers=min(6, len(names))) as ex:
        for name, res in zip(names, ex.map(run_case, names)):
            print(name, res["status"], res["stats"], f"{res['oracle_seconds']} s", flush=True)
            old[name] = res
    with open(OUT, "w") as fh:
        json.dump(dict(sorted(old.items())), fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
