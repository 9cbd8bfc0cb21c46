"""Tile shapes (bins per integral wave, window rows per strip) change only
how the work is split: every setting, and the autotuner's choice, gives the
same outputs bit for bit. Bad settings are rejected."""
import numpy as np
import pytest

from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

pytestmark = pytest.mark.gpu


def _outputs(plan, buf):
    import torch
    torch.cuda.synchronize()
    bins, ii = buf.bins.cpu().numpy(), buf.ii.cpu().numpy()
    out = [buf.scores.cpu().numpy().view(np.uint32)]
    for l in range(plan.sizes.n_levels):
        out += [hog.level_bins(plan, bins, l), hog.level_planes(plan, ii, l)]
    return out


def _setup(nb, k=1):
    import torch
    desc = hog.make_desc(300, 280, channels=3, n_bins=nb, max_levels=0, scale=1.1,
                         n_templates=k, norm=hog.HOG_NORM_L2)
    plan = hog.Plan(desc)
    lut = hog.hog_lut_build(nb)
    img = torch.from_numpy(inputs.synth_image(300, 280, 3, 5100 + nb).reshape(-1)).cuda()
    tmpl, bias = inputs.synth_templates(k, plan.sizes.feature_dim, 5200 + nb)
    return plan, lut, img, torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda()


@pytest.mark.parametrize("nb", [8, 18])
def test_every_tile_shape_gives_identical_outputs(nb):
    plan, lut, img, tt, bt = _setup(nb)
    buf = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    want = _outputs(plan, buf)
    assert hog.plan_tiles(plan).score_rows > 0  # the strip scorer is in use
    for chunk in range(1, 7):
        for rows in (1, 4, 8, 16, 32):
            hog.set_plan_tiles(plan, chunk, rows)
            t = hog.plan_tiles(plan)
            assert (t.bin_chunk, t.score_rows) == (chunk, rows)
            buf.scores.zero_()
            hog.hog_run(plan, lut, img, tt, bt, buf)
            for x, y in zip(want, _outputs(plan, buf)):
                assert np.array_equal(x, y), (chunk, rows)


def test_autotune_picks_valid_tiles_and_keeps_results():
    plan, lut, img, tt, bt = _setup(18)
    buf = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    want = _outputs(plan, buf)
    t = hog.autotune(plan, lut, img, tt, bt, buf, reps=2)
    assert 2 <= t.bin_chunk <= 6 and t.score_rows in (4, 6, 8, 12, 16, 20, 24, 32)
    t2 = hog.plan_tiles(plan)
    assert (t2.bin_chunk, t2.score_rows) == (t.bin_chunk, t.score_rows)
    buf.scores.zero_()
    hog.hog_run(plan, lut, img, tt, bt, buf)
    for x, y in zip(want, _outputs(plan, buf)):
        assert np.array_equal(x, y)


def test_bad_tiles_are_rejected():
    plan, *_ = _setup(8)
    for chunk, rows in ((0, 16), (7, 16), (4, 0), (4, 65)):
        with pytest.raises(hog.HogError) as e:
            hog.set_plan_tiles(plan, chunk, rows)
        assert e.value.status == hog.HOG_E_INVALID
