"""Kernel timing (hog_timing_*): each call records the kernel names the
header lists for it, once per launch, with positive durations; nothing is
recorded while timing is off; a reset clears the totals."""
import numpy as np
import pytest

from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

pytestmark = pytest.mark.gpu

NAMES = ("bin_map", "integral_reduce", "integral_scan", "integral_emit", "integral_soft", "cells",
         "score", "block_features", "score_prep")


def _setup(w=300, h=260, **kw):
    import torch
    desc = hog.make_desc(w, h, channels=3, n_bins=9, max_levels=0, scale=1.2, norm=hog.HOG_NORM_L2, **kw)
    plan = hog.Plan(desc)
    lut = hog.hog_lut_build(9)
    img = torch.from_numpy(inputs.synth_image(w, h, 3, 9100).reshape(-1)).cuda()
    tmpl, bias = inputs.synth_templates(desc.n_templates, plan.sizes.feature_dim, 9101)
    return (plan, lut, img, torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda(),
            hog.Buffers(plan))


def _recorded(runs):
    import torch
    torch.cuda.synchronize()
    out = {}
    for n in NAMES:
        k, ms = hog.hog_timing_get(n)
        if k:
            assert ms > 0.0, n
            out[n] = k
    return out


@pytest.mark.parametrize("kw,want", [
    (dict(), {"bin_map", "integral_reduce", "integral_scan", "integral_emit", "score"}),
    (dict(votes=hog.HOG_VOTES_SOFT), {"bin_map", "integral_soft", "score"}),
    (dict(votes=hog.HOG_VOTES_SOFT, cell=12), {"bin_map", "integral_soft", "cells", "score"}),
    (dict(cell=12), {"bin_map", "integral_reduce", "integral_scan", "integral_emit", "cells", "score"}),
])
def test_each_call_records_its_kernels_once_per_launch(kw, want):
    plan, lut, img, tt, bt, buf = _setup(**kw)
    hog.hog_run(plan, lut, img, tt, bt, buf)  # first use, untimed
    hog.hog_timing_reset()
    hog.hog_timing_enable(True)
    try:
        for _ in range(3):
            hog.hog_run(plan, lut, img, tt, bt, buf)
        got = _recorded(3)
    finally:
        hog.hog_timing_enable(False)
    assert set(got) == want
    assert all(v == 3 for v in got.values()), got


def test_grouped_runs_time_each_group_and_prepare_templates_once():
    plan, lut, img, tt, bt, buf = _setup(640, 480)
    t = hog.plan_tiles(plan)
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 3)
    g = hog.plan_tiles(plan).level_groups
    assert g >= 2
    hog.hog_run(plan, lut, img, tt, bt, buf)
    hog.hog_timing_reset()
    hog.hog_timing_enable(True)
    try:
        for _ in range(2):
            hog.hog_run(plan, lut, img, tt, bt, buf)
        got = _recorded(2)
    finally:
        hog.hog_timing_enable(False)
    assert got["score_prep"] == 2
    for n in ("bin_map", "integral_reduce", "integral_scan", "integral_emit", "score"):
        assert got[n] == 2 * g, (n, got)


def test_nothing_is_recorded_while_off_and_reset_clears():
    plan, lut, img, tt, bt, buf = _setup()
    hog.hog_timing_enable(True)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    hog.hog_timing_enable(False)
    assert _recorded(1)
    hog.hog_timing_reset()
    hog.hog_run(plan, lut, img, tt, bt, buf)
    assert _recorded(1) == {}
    assert hog.hog_timing_get("no_such_kernel") == (0, 0.0)
