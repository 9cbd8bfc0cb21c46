"""The autotune cache on the GPU: the first autotune of a plan shape times
the candidates and stores the result; later ones, in this process or after
the file is read again, install it without timing and leave the buffers as a
tuned call does (their scores equal a hog_run's bit for bit); another shape
is tuned on its own."""
import numpy as np
import pytest
import torch

from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _closed():
    yield
    hog.tune_cache_open(None)


def _tune(desc, seed):
    plan = hog.Plan(desc)
    lut = hog.hog_lut_build(desc.n_bins)
    buf = hog.Buffers(plan)
    img = torch.from_numpy(inputs.synth_image(desc.width, desc.height, desc.channels, seed).reshape(-1)).cuda()
    tmpl, bias = inputs.synth_templates(desc.n_templates, plan.sizes.feature_dim, seed + 1)
    tmpl_t, bias_t = torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda()
    t = hog.autotune(plan, lut, img, tmpl_t, bias_t, buf, reps=1)
    torch.cuda.synchronize()
    tuned = buf.scores.cpu().numpy()[:plan.sizes.score_elems].copy()
    hog.hog_run(plan, lut, img, tmpl_t, bias_t, buf)
    torch.cuda.synchronize()
    again = buf.scores.cpu().numpy()[:plan.sizes.score_elems]
    assert np.array_equal(tuned.view(np.uint32), again.view(np.uint32))
    return (t.bin_chunk, t.score_rows, t.level_groups, t.lut_global)


def test_autotune_results_are_stored_and_reused(tmp_path):
    path = tmp_path / "tiles.txt"
    hog.tune_cache_open(str(path))
    a = hog.make_desc(640, 480, channels=3, n_bins=18, max_levels=0, scale=1.05, norm=hog.HOG_NORM_L2)
    b = hog.make_desc(320, 240, channels=1, n_bins=8, norm=hog.HOG_NORM_RAW)
    ta = _tune(a, 9100)
    assert hog.tune_cache_stats() == (0, 1, 1)
    assert len(path.read_text().splitlines()) == 1
    assert _tune(a, 9102) == ta  # same shape, other image: a hit
    assert hog.tune_cache_stats() == (1, 1, 1)
    _tune(b, 9104)  # another shape: a miss
    assert hog.tune_cache_stats() == (1, 2, 2)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and all(ln.startswith("hogtune ") for ln in lines)
    # As in a new process: the file read again.
    hog.tune_cache_open(str(path))
    assert hog.tune_cache_stats() == (0, 0, 2)
    assert _tune(a, 9106) == ta
    assert hog.tune_cache_stats() == (1, 0, 2)
    assert len(path.read_text().splitlines()) == 2
