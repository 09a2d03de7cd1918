"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Everything on the correction path is comparisons plus one fused multiply-add per edit, so the
required agreement is bit-exact: gradient pairs, critical cell ids, separatrix sequences and
terminals, manifold labels, corrected field bits, quantized edit counts, lossless edits,
statistics and the per-iteration log.
"""
import numpy as np
import pytest

import oracle
from floorcheck import explained
from paper_2409_17346_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _shape3(shape):
    return (shape[1], shape[0], 1) if len(shape) == 2 else (shape[2], shape[1], shape[0])


GRAD_SHAPES = [(2, 2), (3, 3), (7, 5), (33, 65), (130, 67), (2, 2, 2), (5, 4, 3), (9, 17, 6), (31, 12, 20)]


@pytest.mark.parametrize("shape", GRAD_SHAPES)
@pytest.mark.parametrize("kind", ["uniform", "plateau", "const", "perm", "smooth"])
def test_gradient_pairs(ctx, dmt, shape, kind):
    f = synth.random_field(shape, kind, 3)
    up, down, counts = dmt.dmt_gradient_pairs(ctx, _t(f))
    cx = oracle.Complex.grid(*_shape3(shape))
    oup, odn = oracle.gradient(cx, f.reshape(-1))
    assert np.array_equal(up.cpu().numpy(), np.concatenate(oup))
    assert np.array_equal(down.cpu().numpy(), np.concatenate(odn))


MSC_SHAPES = [(3, 3), (16, 9), (64, 64), (129, 70), (3, 3, 3), (8, 7, 6), (17, 20, 13)]


@pytest.mark.parametrize("shape", MSC_SHAPES)
@pytest.mark.parametrize("kind", ["uniform", "plateau", "smooth"])
def test_msc(ctx, dmt, shape, kind):
    f = synth.random_field(shape, kind, 5)
    m = dmt.dmt_extract_msc(ctx, _t(f))
    cx = oracle.Complex.grid(*_shape3(shape))
    o = oracle.msc(cx, f.reshape(-1))
    for d in range(cx.top + 1):
        assert np.array_equal(m[f"crit{d}"].cpu().numpy(), o.crit[d]), d
    pairs = {"desc_saddle": o.desc_saddle, "desc_offsets": o.desc_offsets, "desc_cells": o.desc_cells,
             "desc_terminal": o.desc_terminal, "asc_saddle": o.asc_saddle, "asc_offsets": o.asc_offsets,
             "asc_cells": o.asc_cells, "asc_terminal": o.asc_terminal, "min_label": o.min_label,
             "max_label": o.max_label}
    for k, v in pairs.items():
        assert np.array_equal(m[k].cpu().numpy(), v), k


def test_bounds_and_xi(ctx, dmt):
    rng = np.random.default_rng(2)
    f = np.concatenate([rng.uniform(-3, 3, 5000), rng.uniform(-1e-5, 1e-5, 1000), [0.0, -0.0, 1e-4]]).astype(np.float32)
    for xi in (1e-4, 0.37, 3e-39, 1.0):
        lo, hi = dmt.dmt_bounds(ctx, _t(f), xi)
        olo, ohi = oracle.bounds(f, xi)
        assert np.array_equal(lo.cpu().numpy().view(np.uint32), olo.view(np.uint32))
        assert np.array_equal(hi.cpu().numpy().view(np.uint32), ohi.view(np.uint32))
    g = synth.random_field((40, 30), "smooth", 1)
    for rel in (1e-3, 1e-4, 0.25):
        assert dmt.dmt_xi_from_relative(ctx, _t(g), rel) == synth.xi_from_relative(g, rel)


def _compare_correction(ctx, dmt, w, tier=None, q_max=None, max_iters=-1, flags=0):
    tier = w.tier if tier is None else tier
    q_max = w.q_max if q_max is None else q_max
    nx, ny, nz = w.dims
    cx = oracle.Complex.grid(nx, ny, nz)
    o = oracle.correct(cx, w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, tier, q_max,
                       max_iters=(1 << 40) if max_iters < 0 else max_iters,
                       saddle_saddle=bool(flags & dmt.DMT_F_SADDLE_SADDLE))
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, tier, q_max, max_iters, flags=flags)
    assert r.status == o["status"]
    for k, v in o["stats"].items():
        if k != "status":
            assert r.stats[k] == v, k
    assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32))
    assert np.array_equal(r.q.cpu().numpy().reshape(-1), o["q"])
    assert np.array_equal(r.lossless_idx.cpu().numpy(), o["lossless_idx"])
    assert np.array_equal(r.lossless_val.cpu().numpy().view(np.uint32), o["lossless_val"].view(np.uint32))
    assert np.array_equal(r.log.numpy()[:, :13], o["log"][:, :13])
    assert np.array_equal(r.log.numpy()[:, 20], o["log"][:, 13])     # saddle-saddle troublemakers
    # decoder reproduces the corrected field
    dec = dmt.dmt_apply_edits(ctx, _t(w.g_hat), r.q, r.lossless_idx, r.lossless_val, w.xi, q_max)
    assert torch.equal(dec.view(torch.int32), r.g.view(torch.int32))
    return r, o


CORR_CASES = [
    ((12, 9), "uniform", "noise", 0.2), ((12, 9), "plateau", "bin", 0.2), ((33, 17), "smooth", "noise", 0.05),
    ((64, 48), "uniform", "bin", 0.01), ((5, 4, 3), "uniform", "noise", 0.2), ((9, 8, 7), "plateau", "bin", 0.1),
    ((12, 10, 9), "smooth", "noise", 0.02), ((20, 3, 11), "uniform", "bin", 0.05),
]


FORMS = pytest.mark.parametrize("flags", [0, 1, 2], ids=["persistent", "dense", "phases"])


@pytest.mark.parametrize("shape,kind,ghat,rel", CORR_CASES)
@pytest.mark.parametrize("tier", [1, 2, 3, 4])
@FORMS
def test_correct_small(ctx, dmt, shape, kind, ghat, rel, tier, flags):
    w = synth.tiny_cases(11, shape, rel=rel, kind=kind, ghat=ghat)
    _compare_correction(ctx, dmt, w, tier=tier, flags=flags)


@pytest.mark.parametrize("q_max", [0, 2, 7])
def test_correct_qmax(ctx, dmt, q_max):
    w = synth.tiny_cases(4, (24, 21), rel=0.1, kind="uniform", ghat="noise")
    _compare_correction(ctx, dmt, w, q_max=q_max)


@pytest.mark.parametrize("max_iters", [0, 1, 5, 37])
@FORMS
def test_correct_iteration_cap(ctx, dmt, max_iters, flags):
    w = synth.tiny_cases(6, (30, 20), rel=0.2, kind="uniform", ghat="noise")
    r, o = _compare_correction(ctx, dmt, w, max_iters=max_iters, flags=flags)
    assert r.status == "not_converged" and r.stats["residual_violations"] > 0


@FORMS
def test_correct_small2d_config(ctx, dmt, flags):
    """The 128x128 Gaussian field with 2*xi bins, full MSC (tier 4)."""
    w = synth.config_small2d()
    r, o = _compare_correction(ctx, dmt, w, flags=flags)
    assert r.status == "ok"


@pytest.mark.parametrize("flags", [0, 2], ids=["persistent", "phases"])
def test_correct_large2d_crop(ctx, dmt, flags):
    """A 256x256 corner of the 2048^2 workload (hundreds of C and S iterations)."""
    w = synth.config_large2d()
    w.f = np.ascontiguousarray(w.f[:256, :256])
    w.g_hat = np.ascontiguousarray(w.g_hat[:256, :256])
    r, o = _compare_correction(ctx, dmt, w, flags=flags)
    assert r.status == "ok" and r.stats["s_iterations"] > 100


@pytest.mark.parametrize("limit", [1, 8, 64])
@pytest.mark.parametrize("case", ["small2d", "tiny3d", "crop2d"])
def test_correct_hybrid_handoff(ctx, dmt, limit, case):
    """Iterations with more affected + listed anchors than the limit leave the resident loop for
    full-grid launches and come back: results and log stay those of the oracle."""
    if case == "small2d":
        w = synth.config_small2d()
    elif case == "tiny3d":
        w = synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth", ghat="noise")
    else:
        w = synth.config_large2d()
        w.f = np.ascontiguousarray(w.f[:96, :128])
        w.g_hat = np.ascontiguousarray(w.g_hat[:96, :128])
    dmt.dmt_set_tuning(ctx, {"loop_threads": [1024, 512], "handoff_anchors": [limit, limit],
                             "grid_iterations": [4, 64]})
    try:
        r, o = _compare_correction(ctx, dmt, w)
    finally:
        dmt.dmt_set_tuning(ctx, None)
    log = r.log.numpy()
    assert (log[:, 14] + log[:, 15] > limit).any(), "the hand-off was not exercised"


@pytest.mark.parametrize("flags", [0, 2], ids=["handoff", "phases"])
@pytest.mark.parametrize("case", ["extreme64", "extreme64-tier2", "tiny3d", "atoms3d40"])
def test_correct_dense_iterations(ctx, dmt, case, flags):
    """With every iteration on the full grid (hand-off limit 1, or the per-phase form), the
    iterations whose lists cover more than a quarter of the grid run densely (every vertex dirty,
    every anchor classified by the streaming pass, which also scans every branch from tier 3),
    and a dense iteration after one that edited more than 1/32 of the vertices makes no lists (its
    successor is dense too): results and log stay those of the oracle, and the log shows both
    kinds."""
    tier = None
    if case.startswith("extreme64"):
        w = synth.extreme_noise2d(64, 1)
        tier = 2 if case.endswith("tier2") else None
    elif case == "tiny3d":
        w = synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth", ghat="noise")
    else:
        w = synth.config_atoms3d(seed=3, side=40, n_atoms=24)
    dmt.dmt_set_tuning(ctx, {"loop_threads": [1024, 512], "handoff_anchors": [1, 1], "grid_iterations": [4, 64]})
    try:
        r, o = _compare_correction(ctx, dmt, w, tier=tier, flags=flags)
    finally:
        dmt.dmt_set_tuning(ctx, None)
    n = w.f.size
    log = r.log.numpy()
    dense = log[:, 13] == n              # a dense iteration counts every vertex as dirty
    dense[0] = False                     # iteration 0 is dense by construction
    assert dense.any(), "no dense iteration"
    assert (~dense[1:]).any(), "no frontier iteration"
    unmarked = [it for it in range(2, len(log)) if dense[it] and log[it - 1, 12] > n // 32]
    assert unmarked, "no dense iteration without lists"


def _assert_stall_explained(w, g, tier, n_residual):
    """Every violation left at a stall has an equal-floor, both-at-floor pair of vertices ordered
    against f in the closed 1-ring of the cell's highest vertex: decrease-only edits can never
    separate such a pair (fp32 floors f - xi rounded up merge distinct f values where |f - xi| has
    a larger exponent than f)."""
    nx, ny, nz = w.dims
    cx = oracle.Complex.grid(nx, ny, nz)
    f = w.f.reshape(-1)
    res = oracle.residual(cx, f, g, tier)
    assert len(res) == n_residual
    lo, _ = oracle.bounds(f, w.xi)
    ok = explained(w.dims, f, g, lo, res)
    assert ok.all(), res[~ok][:8]
    return len(res)


def test_correct_atoms3d_small(ctx, dmt):
    """A 40^3 version of the 3D density field (24 atoms, 2*xi bins), full MSC.  Near the 1e-4
    background the fp32 floors collide, and this input stalls in the oracle and on the GPU alike;
    every violation left must be explained by a floor collision."""
    w = synth.config_atoms3d(seed=3, side=40, n_atoms=24)
    r, o = _compare_correction(ctx, dmt, w)
    assert r.status == "not_converged" and r.stats["stalled"] == 1
    assert _assert_stall_explained(w, r.g.cpu().numpy().reshape(-1), 4, r.stats["residual_violations"]) > 0


def test_identity_and_errors(ctx, dmt):
    w = synth.tiny_cases(1, (16, 16), rel=0.1)
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.f), w.xi)
    assert r.status == "ok" and r.stats["iterations"] == 0 and r.stats["n_edited"] == 0
    f = _t(w.f)
    with pytest.raises(dmt.DmtError) as e:
        dmt.dmt_correct(ctx, f, f + 1.0, w.xi)
    assert e.value.status == -2
    bad = f.clone()
    bad[3, 3] = float("nan")
    with pytest.raises(dmt.DmtError) as e:
        dmt.dmt_correct(ctx, bad, f, w.xi)
    assert e.value.status == -3
    with pytest.raises(dmt.DmtError) as e:
        dmt.dmt_correct(ctx, f, f, w.xi, tier=7)
    assert e.value.status == -1
    with pytest.raises(dmt.DmtError) as e:
        dmt.dmt_correct(ctx, f[:1], f[:1], w.xi)
    assert e.value.status == -1


# ------------------------------------------------------------------------------------------
# Batched correction: every job equals the oracle and the single-field call

def _batch_jobs():
    jobs = []
    for i, (shape, kind, ghat, rel) in enumerate(CORR_CASES):
        jobs.append(synth.tiny_cases(30 + i, shape, rel=rel, kind=kind, ghat=ghat))
    jobs.append(synth.config_small2d())
    w = synth.config_large2d()
    w.f = np.ascontiguousarray(w.f[:96, :160])
    w.g_hat = np.ascontiguousarray(w.g_hat[:96, :160])
    jobs.append(w)
    jobs.append(synth.config_atoms3d(seed=5, side=24, n_atoms=8))
    return jobs


@pytest.mark.parametrize("tier", [2, 4])
def test_correct_batch_matches_oracle_and_single(ctx, dmt, tier):
    ws = _batch_jobs()
    fields = [(_t(w.f), _t(w.g_hat), w.xi) for w in ws]
    res = dmt.dmt_correct_batch(ctx, fields, tier=tier, q_max=6)
    for w, r in zip(ws, res):
        nx, ny, nz = w.dims
        o = oracle.correct(oracle.Complex.grid(nx, ny, nz), w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, tier, 6)
        assert r.status == o["status"], w.name
        for k, v in o["stats"].items():
            if k != "status":
                assert r.stats[k] == v, (w.name, k)
        assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32)), w.name
        assert np.array_equal(r.q.cpu().numpy().reshape(-1), o["q"]), w.name
        assert np.array_equal(r.lossless_idx.cpu().numpy(), o["lossless_idx"]), w.name
        s = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, tier, 6)
        assert torch.equal(s.g.view(torch.int32), r.g.view(torch.int32)) and torch.equal(s.q, r.q)


@pytest.mark.parametrize("threads", [(1024, 512), (512, 256)], ids=["wg1024-512", "wg512-256"])
def test_correct_batch_concurrent_handoff(ctx, dmt, threads):
    """With a low hand-off limit several jobs of a batch pause together and run their full-grid
    iterations side by side on separate streams: every job still equals the oracle, with either
    choice of loop workgroup sizes."""
    ws = _batch_jobs()
    fields = [(_t(w.f), _t(w.g_hat), w.xi) for w in ws]
    dmt.dmt_set_tuning(ctx, {"loop_threads": list(threads), "handoff_anchors": [8192, 8192], "grid_iterations": [4, 2],
                             "batch_handoff_anchors": [16, 16]})
    try:
        res = dmt.dmt_correct_batch(ctx, fields, tier=4, q_max=6)
    finally:
        dmt.dmt_set_tuning(ctx, None)
    for w, r in zip(ws, res):
        nx, ny, nz = w.dims
        o = oracle.correct(oracle.Complex.grid(nx, ny, nz), w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, 4, 6)
        assert r.status == o["status"], w.name
        for k, v in o["stats"].items():
            if k != "status":
                assert r.stats[k] == v, (w.name, k)
        assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32)), w.name
        assert np.array_equal(r.q.cpu().numpy().reshape(-1), o["q"]), w.name


@pytest.mark.parametrize("threads", [(512, 256), (1024, 512)], ids=["wg512-256", "wg1024-512"])
@pytest.mark.parametrize("limit", [0, 8192])
def test_tuning_keeps_results(ctx, dmt, threads, limit):
    """Every launch shape gives the oracle's results (2D crop with S-iterations, small 3D field)."""
    dmt.dmt_set_tuning(ctx, {"loop_threads": list(threads), "handoff_anchors": [limit, limit],
                             "grid_iterations": [16, 64]})
    try:
        assert dmt.dmt_get_tuning(ctx)["loop_threads"] == list(threads)
        w = synth.config_large2d()
        w.f = np.ascontiguousarray(w.f[:96, :128])
        w.g_hat = np.ascontiguousarray(w.g_hat[:96, :128])
        _compare_correction(ctx, dmt, w)
        _compare_correction(ctx, dmt, synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth", ghat="noise"))
    finally:
        dmt.dmt_set_tuning(ctx, None)


def test_tuning_rejects_bad_values(ctx, dmt):
    before = dmt.dmt_get_tuning(ctx)
    for bad in ({"loop_threads": [256, 512]}, {"loop_threads": [1024, 1024]}, {"handoff_anchors": [-1, 0]},
                {"grid_iterations": [0, 4]}, {"grid_iterations": [4, 5000]}, {"batch_handoff_anchors": [0, -1]}):
        t = {k: list(v) for k, v in before.items()}
        t.update(bad)
        with pytest.raises(dmt.DmtError):
            dmt.dmt_set_tuning(ctx, t)
        assert dmt.dmt_get_tuning(ctx) == before


def test_tuning_keys_left_out_keep_their_values(ctx, dmt):
    """A partial setting changes only the keys it names; None restores the defaults."""
    dmt.dmt_set_tuning(ctx, None)
    default = dmt.dmt_get_tuning(ctx)
    assert default["handoff_anchors"] == [8192, 1024] and default["batch_handoff_anchors"] == [8192, 8192]
    try:
        dmt.dmt_set_tuning(ctx, {"batch_handoff_anchors": [16, 32]})
        t = dmt.dmt_get_tuning(ctx)
        assert t["batch_handoff_anchors"] == [16, 32]
        assert {k: v for k, v in t.items() if k != "batch_handoff_anchors"} == \
            {k: v for k, v in default.items() if k != "batch_handoff_anchors"}
    finally:
        dmt.dmt_set_tuning(ctx, None)
    assert dmt.dmt_get_tuning(ctx) == default


def test_autotuner_picks_a_setting(ctx, dmt):
    from paper_2409_17346_amd import autotune
    w = synth.config_small2d()
    best, table = autotune.tune_single(ctx, _t(w.f), _t(w.g_hat), w.xi, repeats=1)
    try:
        assert dmt.dmt_get_tuning(ctx) == best
        assert len(table) > 4 and min(r["seconds"] for r in table) > 0
    finally:
        dmt.dmt_set_tuning(ctx, None)


def test_correct_batch_isolates_bad_jobs(ctx, dmt):
    good = synth.tiny_cases(3, (20, 18), rel=0.1, kind="uniform")
    bad = synth.tiny_cases(4, (9, 9), rel=0.1, kind="uniform")
    fields = [(_t(good.f), _t(good.g_hat), good.xi), (_t(bad.f), _t(bad.f) + 1.0, bad.xi),
              (_t(good.f), _t(good.g_hat), good.xi)]
    res = dmt.dmt_correct_batch(ctx, fields)
    assert res[1].status == "bound"
    nx, ny, nz = good.dims
    o = oracle.correct(oracle.Complex.grid(nx, ny, nz), good.f.reshape(-1), good.g_hat.reshape(-1), good.xi, 4, 6)
    for r in (res[0], res[2]):
        assert r.status == o["status"]
        assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32))


# ------------------------------------------------------------------------------------------
# Served form: every job of a request stream equals the oracle

def _server_jobs():
    ws = [synth.tiny_cases(50 + i, shape, rel=rel, kind=kind, ghat=ghat)
          for i, (shape, kind, ghat, rel) in enumerate(CORR_CASES)]
    ws.append(synth.config_small2d())
    ws.append(synth.config_atoms3d(seed=7, side=20, n_atoms=6))
    return ws


def _check_against_oracle(w, r):
    nx, ny, nz = w.dims
    o = oracle.correct(oracle.Complex.grid(nx, ny, nz), w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, 4, 6)
    assert r.status == o["status"], w.name
    for k, v in o["stats"].items():
        if k != "status":
            assert r.stats[k] == v, (w.name, k)
    assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32)), w.name
    assert np.array_equal(r.q.cpu().numpy().reshape(-1), o["q"]), w.name
    assert np.array_equal(r.lossless_idx.cpu().numpy(), o["lossless_idx"]), w.name


@pytest.mark.parametrize("budget,max_jobs", [(64 << 30, 64), (1, 64), (64 << 30, 2)])
def test_server_matches_oracle(dmt, budget, max_jobs):
    """All jobs submitted at once; with a 1-byte budget the server admits one job at a time, with
    max_jobs 2 two at a time."""
    ws = _server_jobs()
    srv = dmt.Server(0, hbm_budget_bytes=budget, max_jobs=max_jobs)
    try:
        tickets = [srv.submit(_t(w.f), _t(w.g_hat), w.xi) for w in ws]
        for w, t in zip(ws, tickets):
            _check_against_oracle(w, srv.poll(t, wait=True))
    finally:
        srv.close()


def test_server_continuous_arrivals(ctx, dmt):
    """Jobs arrive while others run (non-blocking polls in between); each equals dmt_correct."""
    ws = _server_jobs()
    srv = dmt.Server(0, max_jobs=4)
    try:
        live, done = {}, {}
        for i, w in enumerate(ws):
            live[srv.submit(_t(w.f), _t(w.g_hat), w.xi)] = i
            for t in list(live):
                r = srv.poll(t)
                if r is not None:
                    done[live.pop(t)] = r
        for t, i in live.items():
            done[i] = srv.poll(t, wait=True)
        for i, w in enumerate(ws):
            s = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, 4, 6)
            assert done[i].status == s.status and done[i].stats == s.stats, w.name
            assert torch.equal(done[i].g.view(torch.int32), s.g.view(torch.int32)) and torch.equal(done[i].q, s.q)
    finally:
        srv.close()


def test_server_errors(dmt):
    w = synth.tiny_cases(5, (10, 12), rel=0.1, kind="uniform")
    srv = dmt.Server(0)
    try:
        f = _t(w.f)
        with pytest.raises(dmt.DmtError):
            srv.submit(f[:1], f[:1], w.xi)                  # grid too small
        with pytest.raises(dmt.DmtError):
            srv.submit(f, f, w.xi, tier=9)                  # bad tier
        t_bad = srv.submit(f, f + 1.0, w.xi)                # |g_hat - f| > xi
        t_ok = srv.submit(f, _t(w.g_hat), w.xi)
        assert srv.poll(t_bad, wait=True).status == "bound"
        _check_against_oracle(w, srv.poll(t_ok, wait=True))
        with pytest.raises(dmt.DmtError):
            srv.poll(t_ok)                                  # released
    finally:
        srv.close()


def test_server_error_path_frees_each_slot_once(dmt, monkeypatch):
    """A failure in one job's output step (injected) ends the jobs the worker still holds with that
    status, hands every slot back exactly once, and leaves a server that still serves correctly."""
    monkeypatch.setenv("DMT_FAULT_OUTPUTS", "1")
    ws = _server_jobs()
    srv = dmt.Server(0, max_jobs=4)
    try:
        tickets = [srv.submit(_t(w.f), _t(w.g_hat), w.xi) for w in ws]
        res = [srv.poll(t, wait=True) for t in tickets]
        assert sum(r.status == "nomem" for r in res) >= 1
        for w, r in zip(ws, res):
            if r.status != "nomem":
                _check_against_oracle(w, r)
        info = srv.info()
        assert info["free_slots"] == 4 and info["distinct_free_slots"] == 4 and info["pending"] == 0
        # with no job in flight, every accounted byte is memory the idle slots still hold
        assert info["inflight_bytes"] == info["held_bytes"]
        w = ws[-2]
        _check_against_oracle(w, srv.poll(srv.submit(_t(w.f), _t(w.g_hat), w.xi), wait=True))
    finally:
        srv.close()


def test_server_budget_accounting(dmt):
    """With a budget below two jobs' footprints the jobs of a burst run one at a time, each equal to
    the oracle; once the server is idle every accounted byte is memory its slots still hold."""
    ws = _server_jobs()[-3:]
    est = max(dmt.dmt_workspace_bytes(w.f.shape) for w in ws)
    srv = dmt.Server(0, hbm_budget_bytes=est + (est // 2), max_jobs=8)
    try:
        tickets = [srv.submit(_t(w.f), _t(w.g_hat), w.xi) for w in ws]
        for w, t in zip(ws, tickets):
            _check_against_oracle(w, srv.poll(t, wait=True))
        info = srv.info()
        assert info["inflight_bytes"] == info["held_bytes"] > 0
        assert info["free_slots"] == info["distinct_free_slots"] == 8
    finally:
        srv.close()


def test_lossless_list_matches_correct(ctx, dmt):
    """dmt_lossless_list reads a job's lossless edits from q_out and g_out: the same list that
    dmt_correct keeps in the context."""
    w = synth.config_small2d()
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi)
    idx, val = dmt.dmt_lossless_list(ctx, r.q, r.g)
    assert r.lossless_idx.numel() > 0
    assert torch.equal(idx, r.lossless_idx) and torch.equal(val.view(torch.int32), r.lossless_val.view(torch.int32))


AGREE_CASES = [((12, 9), "uniform", 0.2), ((64, 48), "smooth", 0.01), ((130, 67), "plateau", 0.05),
               ((5, 4, 3), "uniform", 0.2), ((12, 10, 9), "smooth", 0.02), ((20, 17, 19), "plateau", 0.05)]


@pytest.mark.parametrize("shape,kind,rel", AGREE_CASES)
def test_compare_msc(ctx, dmt, shape, kind, rel):
    """Critical-cell and separatrix agreement counts (the recall / precision of Section 5.1) equal
    the oracle's, for g_hat and for the fields corrected at tiers 2 and 4."""
    w = synth.tiny_cases(7, shape, rel=rel, kind=kind, ghat="noise")
    cx = oracle.Complex.grid(*w.dims)
    f = w.f.reshape(-1)
    for tier in (0, 2, 4):
        status = "ok"
        if tier == 0:
            g = w.g_hat
        else:
            r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, tier, 6)
            g, status = r.g.cpu().numpy(), r.status
        a = dmt.dmt_compare_msc(ctx, _t(w.f), _t(g))
        o = oracle.msc_agreement(cx, f, g.reshape(-1))
        for k, v in o.items():
            assert a[k] == v, (tier, k)
        if tier == 4 and status == "ok":
            assert a["critical_recall"] == a["critical_precision"] == 1.0
            assert a["separatrix_recall"] == 1.0


def test_compare_msc_small2d_config(ctx, dmt):
    w = synth.config_small2d()
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, 4, 6)
    cx = oracle.Complex.grid(*w.dims)
    for g in (w.g_hat, r.g.cpu().numpy()):
        a = dmt.dmt_compare_msc(ctx, _t(w.f), _t(g))
        o = oracle.msc_agreement(cx, w.f.reshape(-1), g.reshape(-1))
        for k, v in o.items():
            assert a[k] == v, k
    assert a["separatrix_recall"] == a["separatrix_precision"] == a["critical_recall"] == 1.0


@pytest.mark.parametrize("q_max", range(8))
def test_edit_stream_random(ctx, dmt, q_max):
    """The packed stream equals the oracle's bit for bit (codes straddling words, ragged tails);
    the decoder returns the counts."""
    rng = np.random.default_rng(100 + q_max)
    for n in (1, 33, 4099, 70001):
        q = rng.integers(0, q_max + 2, size=n).astype(np.uint8)
        q[q == q_max + 1] = 0xFF
        g = rng.uniform(0, 1, size=n).astype(np.float32)
        stream, val = dmt.dmt_pack_edits(ctx, _t(q, torch.uint8), _t(g), q_max)
        assert np.array_equal(stream.cpu().numpy().view(np.uint32), oracle.pack_edits(q, q_max))
        assert np.array_equal(val.cpu().numpy().view(np.uint32), g[q == 0xFF].view(np.uint32))
        gh = rng.uniform(0, 1, size=n).astype(np.float32)
        xi = 0.01
        g2, q2 = dmt.dmt_unpack_edits(ctx, stream, val, _t(gh), xi, q_max)
        assert np.array_equal(q2.cpu().numpy(), q)
        ref = oracle.decode(gh, q, np.nonzero(q == 0xFF)[0], g[q == 0xFF], xi, q_max)
        assert np.array_equal(g2.cpu().numpy().view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("case", ["small2d", "tiny3d"])
def test_edit_stream_of_a_correction(ctx, dmt, case):
    """dmt_correct -> stream + lossless values -> DEFLATE -> inflate -> decoder gives g' bit for bit."""
    w = synth.config_small2d() if case == "small2d" else synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth",
                                                                          ghat="noise")
    r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, 4, w.q_max)
    stream, val = dmt.dmt_pack_edits(ctx, r.q, r.g, w.q_max)
    assert val.numel() == r.stats["n_lossless"]
    assert torch.equal(val.view(torch.int32), r.lossless_val.view(torch.int32))
    blob = dmt.compress_edits(stream, val)
    s2, v2 = dmt.decompress_edits(blob)
    g2, q2 = dmt.dmt_unpack_edits(ctx, s2, v2, _t(w.g_hat), w.xi, w.q_max)
    assert torch.equal(g2.view(torch.int32), r.g.view(torch.int32)) and torch.equal(q2, r.q)


def test_edit_stream_errors(ctx, dmt):
    q = torch.zeros(100, dtype=torch.uint8, device="cuda")
    g = torch.zeros(100, device="cuda")
    q[5] = 9                                   # above q_max = 6 and not the lossless marker
    with pytest.raises(dmt.DmtError):
        dmt.dmt_pack_edits(ctx, q, g, 6)
    q[5] = 0xFF
    stream, val = dmt.dmt_pack_edits(ctx, q, g, 6)
    with pytest.raises(dmt.DmtError):         # one lossless vertex marked, none given
        dmt.dmt_unpack_edits(ctx, stream, val[:0], g, 0.1, 6)
    bad = torch.full(((100 * 4 + 31) // 32,), -1, dtype=torch.int32, device="cuda")
    with pytest.raises(dmt.DmtError) as e:     # every 4-bit code of q_max 7 reads 15 > 8
        dmt.dmt_unpack_edits(ctx, bad, val, g, 0.1, 7)
    assert "code above" in str(e.value)


@pytest.mark.parametrize("side", [64, 100, 128])
def test_extreme_flat_noise(ctx, dmt, side):
    """The extreme case (noise in [0, xi), flat g_hat): oracle's results bit for bit."""
    r, o = _compare_correction(ctx, dmt, synth.extreme_noise2d(side, 1))
    assert r.status == "ok" and r.stats["n_edited"] > side * side // 3


@pytest.mark.parametrize("q_max", range(2, 8))
@pytest.mark.parametrize("rel", [1e-4, 1e-3])
def test_qmax_sweep_field(ctx, dmt, q_max, rel):
    """The q_max sweep's 150 x 450 field: oracle's results for every q_max."""
    _compare_correction(ctx, dmt, synth.flow2d(150, 450, 3, rel), q_max=q_max)


@pytest.mark.parametrize("tier", [1, 2, 3, 4])
def test_tier_study_field(ctx, dmt, tier):
    """The tier study's 361 x 576 field: oracle's results at every tier, and the agreement each
    tier guarantees."""
    w = synth.flow2d(361, 576, 4, 1e-4)
    r, o = _compare_correction(ctx, dmt, w, tier=tier)
    a = dmt.dmt_compare_msc(ctx, _t(w.f), r.g)
    if tier >= 2:
        assert a["critical_recall"] == a["critical_precision"] == 1.0
    if tier >= 3:
        assert a["separatrix_recall_connectivity"] == 1.0
    if tier == 4:
        assert a["separatrix_recall"] == a["separatrix_precision"] == 1.0


SS_GPU_CASES = [((4, 4, 5), "smooth", 0), ((4, 5, 5), "smooth", 4), ((4, 5, 6), "uniform", 6),
                ((4, 5, 6), "smooth", 10), ((9, 10, 12), "smooth", 13), ((17, 11, 23), "uniform", 2)]


@pytest.mark.parametrize("shape,kind,seed", SS_GPU_CASES)
@FORMS
def test_saddle_saddle(ctx, dmt, shape, kind, seed, flags):
    """Tier 4 with saddle-saddle connectors (3D): the oracle's results and log in every form."""
    w = synth.tiny_cases(seed, shape, rel=0.2 if max(shape) < 8 else 0.05, kind=kind, ghat="noise")
    r, o = _compare_correction(ctx, dmt, w, tier=4, flags=flags | dmt.DMT_F_SADDLE_SADDLE)
    if max(shape) < 8:
        assert o["log"][:, 13].sum() > 0


@pytest.mark.parametrize("case", ["lognormal32", "lognormal48"])
def test_saddle_saddle_fields(ctx, dmt, case):
    w = synth.lognormal_case(32, 3) if case == "lognormal32" else synth.lognormal_case(48, 4)
    r, o = _compare_correction(ctx, dmt, w, tier=4, flags=dmt.DMT_F_SADDLE_SADDLE)
    assert r.status == "ok" and o["log"][:, 13].sum() > 0


@pytest.mark.parametrize("limit", [1, 64])
def test_saddle_saddle_handoff(ctx, dmt, limit):
    """Saddle-saddle walks in the full-grid hand-off iterations (a one-workgroup launch)."""
    w = synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth", ghat="noise")
    dmt.dmt_set_tuning(ctx, {"loop_threads": [1024, 512], "handoff_anchors": [limit, limit],
                             "grid_iterations": [4, 64]})
    try:
        _compare_correction(ctx, dmt, w, tier=4, flags=dmt.DMT_F_SADDLE_SADDLE)
    finally:
        dmt.dmt_set_tuning(ctx, None)


def test_saddle_saddle_batch_and_2d(ctx, dmt):
    """The option in a batch (3D jobs walk their connectors, 2D jobs are unchanged)."""
    ws = [synth.tiny_cases(13, (12, 10, 9), rel=0.05, kind="smooth", ghat="noise"),
          synth.tiny_cases(0, (4, 4, 5), rel=0.2, kind="smooth", ghat="noise"), synth.config_small2d()]
    res = dmt.dmt_correct_batch(ctx, [(_t(w.f), _t(w.g_hat), w.xi) for w in ws], tier=4,
                                flags=dmt.DMT_F_SADDLE_SADDLE)
    for w, r in zip(ws, res):
        o = oracle.correct(oracle.Complex.grid(*w.dims), w.f.reshape(-1), w.g_hat.reshape(-1), w.xi, 4, 6,
                           saddle_saddle=True)
        assert r.status == o["status"]
        assert np.array_equal(r.g.cpu().numpy().reshape(-1).view(np.uint32), o["g"].view(np.uint32)), w.name
