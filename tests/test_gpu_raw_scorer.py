"""Raw-feature window scores (Sec. 3.1 / Fig. 4, Sec. 4): the feature is the
window's cell histograms in row-major order, the score its inner product with
the template plus the bias. Every window of every level is compared with the
oracle (FP64, cells counted by brute force) within 1e-5 (sum |T f| + |b|).

The cases reach each form of the raw scorer: 64-window tiles with the bin
count and window width fixed at compile time (N_b 8, 9, 18 in 8-cell-wide
windows) and at run time (other bin counts and widths), waves that take one
cell row or several (windows 12 and 20 cells high), template counts of 1, 2
and 3 (the cross-wave sums alternate between two LDS buffers), tiles cut by the
level's edge (one window column), cells of 12 pixels (cells from the planes),
soft votes, and 64 bins, whose tiles do not fit LDS and go to the older
vector scorer."""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_params, run_gpu, templates_for

pytestmark = pytest.mark.gpu

# (width, height, channels, n_bins, K, max_levels, scale, scan overrides)
CASES = [
    (320, 240, 1, 8, 1, 1, 1.0, {}),
    (400, 300, 3, 9, 3, 0, 1.1, {}),
    (260, 200, 1, 18, 2, 2, 1.1, {}),
    (300, 220, 1, 12, 1, 1, 1.0, {}),
    (250, 270, 1, 8, 2, 1, 1.0, dict(win_cells_x=6, win_cells_y=12)),
    (200, 260, 1, 8, 1, 1, 1.0, dict(win_cells_x=4, win_cells_y=20)),
    (64, 300, 1, 8, 2, 1, 1.0, {}),
    (300, 300, 1, 8, 1, 1, 1.0, dict(cell=12)),
    (200, 200, 1, 64, 1, 1, 1.0, {}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_raw_scores_every_window(case):
    w, h, c, nb, k, levels, scale, scan = CASES[case]
    desc = hog.make_desc(w, h, channels=c, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_RAW,
                         max_levels=levels, scale=scale, **scan)
    img = inputs.synth_image(w, h, c, 8100 + case)
    tmpl, bias = templates_for(desc, 8150 + case)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    p = oracle_params(desc)
    n = 0
    for l, li in enumerate(plan.levels):
        if li.windows_x == 0:
            continue
        lvl = img if l == 0 else oracle.resize_nn(img, li.scale, li.width, li.height)
        bins = oracle.bin_map(lvl, nb)
        ref, absterm, _, wxs, wys = oracle.score_windows(bins, nb, p, tmpl, bias)
        check_scores(hog.level_scores(plan, out["scores"], l)[wys, wxs, :], ref, absterm)
        n += len(wxs)
    assert n > 0


def test_raw_scores_soft_votes():
    w, h, nb, k = 320, 240, 8, 2
    desc = hog.make_desc(w, h, channels=1, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_RAW,
                         votes=hog.HOG_VOTES_SOFT)
    img = inputs.synth_image(w, h, 1, 8190)
    tmpl, bias = templates_for(desc, 8191)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    li = plan.levels[0]
    b0, w1 = oracle.soft_bin_map(img, nb)
    idx = np.arange(li.windows_x * li.windows_y)
    ref, absterm, wxs, wys = oracle.soft_score_windows(b0, w1, nb, oracle_params(desc), tmpl, bias,
                                                       idx % li.windows_x, idx // li.windows_x)
    check_scores(hog.level_scores(plan, out["scores"], 0)[wys, wxs, :], ref, absterm)


def test_raw_scores_repeat_bit_identical():
    """Two runs on the same buffers give the same scores bit for bit (the
    per-window FP64 sums have a fixed order)."""
    desc = hog.make_desc(320, 240, channels=1, n_bins=8, n_templates=3, norm=hog.HOG_NORM_RAW)
    img = inputs.synth_image(320, 240, 1, 8195)
    tmpl, bias = templates_for(desc, 8196)
    _, outs = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False, repeat=2)
    n = hog.Plan(desc).sizes.score_elems
    assert np.array_equal(outs[0]["scores"][:n].view(np.uint32), outs[1]["scores"][:n].view(np.uint32))
