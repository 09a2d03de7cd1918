"""The allocation-free correction (dmt_correct_noalloc) against dmt_correct, through the C ABI.

Both entry points run the same kernels; the allocation-free one carves every buffer from the
library's per-device scratch array.  Its results must equal dmt_correct's bit for bit, on
consecutive calls of shrinking size (the scratch keeps the previous call's contents), and the
context must keep working for ordinary calls afterwards.
"""
import numpy as np
import pytest

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


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _cases():
    big = synth.config_large2d()
    big.f = np.ascontiguousarray(big.f[:256, :256])
    big.g_hat = np.ascontiguousarray(big.g_hat[:256, :256])
    small = synth.config_small2d()
    cube = synth.config_atoms3d(seed=5, side=24, n_atoms=8)
    return [big, small, cube]


def _same(r, ref):
    assert r.status == ref.status
    assert r.stats == ref.stats
    assert torch.equal(r.g.view(torch.int32), ref.g.view(torch.int32))
    assert torch.equal(r.q, ref.q)
    assert torch.equal(r.lossless_idx, ref.lossless_idx)
    assert torch.equal(r.lossless_val.view(torch.int32), ref.lossless_val.view(torch.int32))


def _noalloc(dmt, ctx, w, cap=None, tier=4):
    f, gh = _t(w.f), _t(w.g_hat)
    cap = f.numel() if cap is None else cap
    g_out = torch.full_like(f, float("nan"))
    q_out = torch.full(f.shape, 0x55, dtype=torch.uint8, device="cuda")
    idx = torch.full((cap,), -7, dtype=torch.int64, device="cuda")
    val = torch.full((cap,), float("nan"), device="cuda")
    return dmt.dmt_correct_noalloc(ctx, f, gh, w.xi, g_out, q_out, idx, val, tier=tier, q_max=w.q_max)


def test_noalloc_matches_correct_on_consecutive_calls(dmt):
    ref_ctx = dmt.Context(0)
    ctx = dmt.Context(0)
    try:
        for w in _cases():                       # 65536, then 16384, then 13824 vertices
            print(f"[no_alloc] {w.name} {w.f.shape}", flush=True)
            ref = dmt.dmt_correct(ref_ctx, _t(w.f), _t(w.g_hat), w.xi, 4, w.q_max)
            r = _noalloc(dmt, ctx, w)
            torch.cuda.synchronize()
            _same(r, ref)
            assert r.stats["n_lossless"] == r.lossless_idx.numel()
        # the context still serves ordinary calls, with its own buffers
        w = _cases()[1]
        ref = dmt.dmt_correct(ref_ctx, _t(w.f), _t(w.g_hat), w.xi, 3, w.q_max)
        r = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, 3, w.q_max)
        _same(r, ref)
        assert torch.equal(r.log[:, :19], ref.log[:, :19])   # word 19 is a duration
    finally:
        ctx.close()
        ref_ctx.close()


def test_noalloc_limits(dmt):
    ctx = dmt.Context(0)
    try:
        # a lossless list longer than the destination: error, with the count reported
        w = _cases()[1]
        ref = dmt.dmt_correct(ctx, _t(w.f), _t(w.g_hat), w.xi, 4, w.q_max)
        n_ll = ref.stats["n_lossless"]
        assert n_ll > 1
        with pytest.raises(dmt.DmtError) as e:
            _noalloc(dmt, ctx, w, cap=n_ll - 1)
        assert e.value.status == dmt.DMT_E_INVALID
        r = _noalloc(dmt, ctx, w, cap=n_ll)
        _same(r, ref)
        # fields whose workspace exceeds the scratch are refused before any work
        side = 1000                              # 1.0 M vertices: 144 B each exceeds 128 MiB
        big = torch.zeros((side, side), device="cuda")
        assert dmt.dmt_workspace_bytes((side, side)) > dmt.DMT_NOALLOC_SCRATCH_BYTES
        with pytest.raises(dmt.DmtError) as e:
            dmt.dmt_correct_noalloc(ctx, big, big, 1e-3, torch.empty_like(big),
                                    torch.empty(big.shape, dtype=torch.uint8, device="cuda"),
                                    torch.empty(1, dtype=torch.int64, device="cuda"),
                                    torch.empty(1, device="cuda"))
        assert e.value.status == dmt.DMT_E_NOMEM
        assert "scratch" in str(e.value)
    finally:
        ctx.close()
