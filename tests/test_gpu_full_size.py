"""GPU parity at the workloads' full sizes, in the launch configuration the benchmark times.

The oracle's results on full-size inputs are stored as hashes in tests/golden/full_size.json,
written by tests/golden/make_full_size.py (which calls only the oracle and the seeded input
generators).  Each test regenerates the input, checks that it hashes as stored, runs the HIP path
through the C ABI and compares the hashes of every output: corrected field bits, quantized edit
counts, lossless edit ids and value bits, statistics and the per-iteration log.

The 256^3 density field is beyond the oracle (its explicit complex has 432 M cells); there the
test checks properties that hold at any size: the bound, decrease-only edits, the decoder round
trip, and that every violation left at the stall is a floor collision.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from floorcheck import explained
from paper_2409_17346_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_full_size import CASES, input_hashes, output_hashes  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_GOLDEN_PATH = os.path.join(HERE, "golden", "full_size.json")
GOLDEN = json.load(open(_GOLDEN_PATH)) if os.path.exists(_GOLDEN_PATH) else {}


@pytest.fixture(scope="module")
def dmt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_17346_amd import dmt as D
    D.load_library()
    return D


@pytest.fixture(scope="module")
def ctx(dmt):
    c = dmt.Context(0)
    yield c
    c.close()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _input(name):
    recipe, tier = CASES[name]
    w = eval(recipe, {"synth": synth})
    g = GOLDEN[name]
    assert input_hashes(w) == g["input"], f"{name}: the generator no longer reproduces the stored input"
    assert tier == g["tier"]
    return w, g


def _check(name, g, status, stats, gout, q, idx, val, log):
    assert status == g["status"], name
    assert stats == g["stats"], name
    log13 = np.zeros((0, 13), np.int64) if log is None else log.numpy()[:, :13]
    got = output_hashes(gout.cpu().numpy(), q.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy(), log13)
    if log is None:
        got["log13"] = g["outputs"]["log13"]     # batch and server keep no per-iteration log
    assert got == g["outputs"], name


SINGLE = ["2d-2048-gauss256-valuenoise-noise-1e-4", "3d-128-lognormal-bin-1e-4"]
BATCH = ["batch0-0-2d-481", "batch0-3-2d-557", "batch0-33-3d-95", "batch0-34-3d-101"]


@pytest.mark.parametrize("name", SINGLE)
def test_full_size_single(ctx, dmt, name):
    if name not in GOLDEN:
        pytest.skip(f"no stored result for {name}")
    w, g = _input(name)
    print(f"[full] {name}", flush=True)
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, g["tier"], g["q_max"])
    stats = {k: int(v) for k, v in r.stats.items()}
    _check(name, g, r.status, stats, r.g, r.q, r.lossless_idx, r.lossless_val, r.log)


def test_full_size_batch_subset(ctx, dmt):
    names = [n for n in BATCH if n in GOLDEN]
    if len(names) < len(BATCH):
        pytest.skip("stored batch results incomplete")
    ws = [_input(n) for n in names]
    print(f"[full] batch of {names}", flush=True)
    res = dmt.dmt_correct_batch(ctx, [(_t(w.f), _t(w.g_hat), w.xi) for w, _ in ws])
    for n, (w, g), r in zip(names, ws, res):
        stats = {k: int(v) for k, v in r.stats.items()}
        _check(n, g, r.status, stats, r.g, r.q, r.lossless_idx, r.lossless_val, None)


def test_full_size_atoms3d_stall_is_floor_collisions(ctx, dmt):
    """256^3 density field: tier 4 stalls; every violation left is an fp32 floor collision."""
    w = synth.config_atoms3d()
    print(f"[full] {w.name}", flush=True)
    f, gh = _t(w.f), _t(w.g_hat)
    r = dmt.dmt_correct(ctx, f, gh, w.xi, 4, 6, want_edits=True)
    assert r.status == "not_converged" and r.stats["stalled"] == 1
    fl = w.f.reshape(-1)
    g = r.g.cpu().numpy().reshape(-1)
    lo, _ = oracle.bounds(fl, w.xi)
    # bound and decrease-only edits, decoder round trip
    assert (g >= lo).all() and (g <= w.g_hat.reshape(-1)).all()
    dec = dmt.dmt_apply_edits(ctx, gh, r.q, r.lossless_idx, r.lossless_val, w.xi, 6)
    assert torch.equal(dec.view(torch.int32), r.g.view(torch.int32))
    # the violations left: cells critical in exactly one of f and g'
    mf = dmt.dmt_extract_msc(ctx, f)
    crit_f = [mf[f"crit{d}"].cpu().numpy() for d in range(4)]
    mg = dmt.dmt_extract_msc(ctx, r.g)
    crit_g = [mg[f"crit{d}"].cpu().numpy() for d in range(4)]
    cells = np.concatenate([np.stack([np.full(len(x), d), x], 1)
                            for d in range(4) for x in [np.setxor1d(crit_f[d], crit_g[d])]])
    assert len(cells) == r.stats["residual_violations"] > 0
    ok = explained(w.dims, fl, g, lo, cells)
    print(f"[full] {w.name}: {len(cells)} residual violations, {int(ok.sum())} floor collisions", flush=True)
    assert ok.all()


def test_tiled_scan_reaches_msc(ctx, dmt):
    """A 512^2 uniform-noise field has > 65536 descending branches, so the separatrix scans run
    tiled; the MSC must still equal the oracle's."""
    f = synth.random_field((512, 512), "uniform", 9)
    m = dmt.dmt_extract_msc(ctx, _t(f))
    assert m["desc_saddle"].numel() > 65536
    o = oracle.msc(oracle.Complex.grid(512, 512, 1), f.reshape(-1))
    for d in range(3):
        assert np.array_equal(m[f"crit{d}"].cpu().numpy(), o.crit[d]), d
    for k in ("desc_saddle", "desc_offsets", "desc_cells", "desc_terminal", "asc_saddle", "asc_offsets",
              "asc_cells", "asc_terminal", "min_label", "max_label"):
        assert np.array_equal(m[k].cpu().numpy(), getattr(o, k)), k
