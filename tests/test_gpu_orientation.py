"""Unsigned orientation (the table variant of Fig. 4's 9-bin, 0..180 degree
example): the host table, and the whole path run with it, against the
oracle's unsigned bins -- bins, planes and cells bit for bit, scores within
tolerance. The kernels are those of the signed path; only the table differs."""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_level_bins, oracle_params, run_gpu, templates_for

pytestmark = pytest.mark.gpu

U = hog.HOG_ORIENT_UNSIGNED


def test_unsigned_host_table_matches_oracle():
    """The host copy of a built unsigned table; the device copies are read
    back in test_gpu_lut_pairs."""
    for nb in (4, 9, 18, 64):
        lut = hog.hog_lut_build(nb, U)
        assert hog.load_library().hog_lut_orientation(lut.handle) == U
        assert np.array_equal(lut.host_table(), oracle.bin_table(nb, unsigned=True))
        lut.free()


@pytest.mark.parametrize("kw", [
    dict(width=320, height=240, channels=1, n_bins=9),
    dict(width=800, height=600, channels=3, n_bins=9, norm=hog.HOG_NORM_L2),
    dict(width=300, height=331, channels=3, n_bins=18, max_levels=0, scale=1.1, norm=hog.HOG_NORM_L2),
    dict(width=200, height=170, channels=3, n_bins=33, norm=hog.HOG_NORM_L2),
    dict(width=640, height=480, channels=3, n_bins=9, n_templates=32, max_levels=3, scale=1.2,
         norm=hog.HOG_NORM_L2),
])
def test_unsigned_path_equals_oracle(kw):
    desc = hog.make_desc(**kw)
    img = inputs.synth_image(kw["width"], kw["height"], kw["channels"], 7700 + kw["n_bins"])
    tmpl, bias = templates_for(desc, 7701)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=True, block_feat=False, orientation=U)
    nb = desc.n_bins
    for l in range(plan.sizes.n_levels):
        li = plan.levels[l]
        want = oracle_level_bins(img, plan, l, unsigned=True)
        assert np.array_equal(hog.level_bins(plan, out["bins"], l), want), f"bins, level {l}"
        assert np.array_equal(hog.level_planes(plan, out["ii"], l), oracle.integral(want, nb)[:, 1:, 1:])
        if li.cells_x and li.cells_y:
            assert np.array_equal(hog.level_cells(plan, out["cells"], l), oracle.cell_hist(want, nb, 8))
        if li.windows_x:
            rng = np.random.default_rng(l)
            n = min(60, li.windows_x * li.windows_y)
            idx = rng.choice(li.windows_x * li.windows_y, size=n, replace=False)
            ref, absterm, _, wxs, wys = oracle.score_windows(want, nb, oracle_params(desc), tmpl, bias,
                                                             idx % li.windows_x, idx // li.windows_x)
            check_scores(hog.level_scores(plan, out["scores"], l)[wys, wxs, :], ref, absterm)


def test_server_with_unsigned_orientation():
    import time
    import torch
    torch.cuda.init()
    K = 4
    desc = hog.make_desc(320, 240, channels=3, n_bins=9, n_templates=K, norm=hog.HOG_NORM_L2)
    tmpl, bias = templates_for(desc, 7800)
    srv = hog.Server(tmpl, bias, channels=3, n_bins=9, max_width=320, max_height=240,
                     memory_budget=128 << 20, orientation=U)
    img = inputs.synth_image(320, 240, 3, 7801)
    t = srv.submit(img)
    t0 = time.time()
    cap = (40 - 7) * (30 - 15) * K
    while (r := srv.poll(t, cap)) is None:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    srv.close()
    _, alone = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False, orientation=U)
    assert np.array_equal(r[0].view(np.uint32), alone["scores"][:cap].view(np.uint32))
