"""Host-only checks of the C ABI library (no GPU needed): it loads, exports every entry point
that include/dmt.h declares, and validates grids without touching a device."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dmt.h")).read()
    return sorted(set(re.findall(r"^\s*(?:dmt_status|const char \*|int64_t|int32_t)\s*(dmt_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2409_17346_amd import dmt
    L = dmt.load_library()
    decl = _declared()
    assert len(decl) >= 13
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(dmt.ABI_SYMBOLS) == decl


def test_cell_id_space_and_validation():
    from paper_2409_17346_amd import dmt
    assert dmt.dmt_cell_id_space((128, 128)) == (16384, 49152, 32768, 0)
    assert dmt.dmt_cell_id_space((4, 5, 6)) == (120, 840, 1440, 720)
    with pytest.raises(dmt.DmtError):
        dmt.dmt_cell_id_space((1, 5))
    with pytest.raises(dmt.DmtError):
        dmt.dmt_cell_id_space((1, 5, 5))
    with pytest.raises(dmt.DmtError):
        dmt.dmt_cell_id_space((2048, 2048, 2048))


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_2409_17346_amd import dmt
    with pytest.raises(ValueError):
        dmt._dev(torch.zeros(4, 4))


def test_workspace_estimate():
    from paper_2409_17346_amd import dmt
    assert dmt.dmt_workspace_bytes((128, 128)) == 144 * 128 * 128 + (1 << 20)
    assert dmt.dmt_workspace_bytes((8, 9, 10)) == 264 * 720 + (1 << 20)
    assert dmt.dmt_workspace_bytes((1, 9)) == -1


def test_noalloc_scratch_size_matches_header():
    from paper_2409_17346_amd import dmt
    src = open(os.path.join(ROOT, "include", "dmt.h")).read()
    m = re.search(r"#define DMT_NOALLOC_SCRATCH_BYTES (\d+)LL", src)
    assert m and int(m.group(1)) == dmt.DMT_NOALLOC_SCRATCH_BYTES


def test_edit_bits():
    from paper_2409_17346_amd import dmt
    L = dmt.load_library()
    assert [L.dmt_edit_bits(q) for q in range(8)] == [1, 2, 2, 3, 3, 3, 3, 4]
    assert L.dmt_edit_bits(-1) == -1 and L.dmt_edit_bits(8) == -1
