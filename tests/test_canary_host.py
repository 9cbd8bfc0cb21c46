"""The guard-band check the GPU tests rely on (hog_cases.GuardedBuffers),
exercised on CPU tensors: untouched guards pass, a byte written just before
or just after a buffer is reported."""
import types

import pytest

import hog_cases


def _plan():
    sizes = types.SimpleNamespace(bins_bytes=1000, ii_elems=333, score_elems=7, workspace_bytes=4096,
                                  cell_elems=20, block_elems=30, ii_elem_bytes=4)
    return types.SimpleNamespace(sizes=sizes, desc=types.SimpleNamespace(plane_bits=32))


@pytest.fixture(autouse=True)
def _ii_dtype(monkeypatch):
    import torch
    monkeypatch.setattr(hog_cases.hog, "ii_dtype", lambda plan: torch.int32)


def test_untouched_guards_pass_and_writes_inside_are_fine():
    b = hog_cases.GuardedBuffers(_plan(), device="cpu", cell_hist=True, block_feat=True)
    b.bins.fill_(1)
    b.ii.fill_(-1)
    b.scores.fill_(3.0)
    b.workspace.fill_(0)
    b.cell_hist.fill_(9)
    b.block_feat.fill_(0.5)
    b.check_guards()
    hog_cases._guarded.clear()


@pytest.mark.parametrize("where", ["before", "after"])
@pytest.mark.parametrize("name", ["bins", "ii", "scores", "workspace", "cell_hist", "block_feat"])
def test_a_write_outside_a_buffer_is_reported(name, where):
    import torch
    b = hog_cases.GuardedBuffers(_plan(), device="cpu", cell_hist=True, block_feat=True)
    for n, base, g, size in b._regions:
        if n == name:
            raw = base.view(torch.uint8)
            raw[g - 1 if where == "before" else g + size] = 0
    with pytest.raises(AssertionError, match=f"{where} the {name} buffer"):
        b.check_guards()
    hog_cases._guarded.clear()
