"""Narrow integral images (plane_bits 16 and 8; Sec. 4's 16-bit integral
images, read mod 2^bits): the planes equal the oracle's exact planes mod
2^bits bit for bit; cell histograms taken from them (four-corner sums mod
2^bits) equal the oracle's brute-force counts, also where the planes wrap;
scores equal those of the same plan with uint32 planes bit for bit (the
scorer reads the same cell cache) and the oracle's within tolerance."""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_level_bins, oracle_params, run_gpu, run_gpu_batch, templates_for

pytestmark = pytest.mark.gpu


def _desc(bits, **kw):
    return hog.make_desc(plane_bits=bits, **kw)


def _check_planes_and_cells(plan, out, img, l, bits, l0=0):
    d = plan.desc
    nb = d.n_bins
    li = plan.levels[l]
    want_bins = oracle_level_bins(img, plan, l, l0)
    assert np.array_equal(hog.level_bins(plan, out["bins"], l), want_bins), f"bins, level {l}"
    got = hog.level_planes(plan, out["ii"], l)
    assert got.dtype == (np.uint16 if bits == 16 else np.uint8)
    want = oracle.integral_mod(want_bins, nb, bits)[:, 1:, 1:]
    assert np.array_equal(got, want), f"planes mod 2^{bits}, level {l}"
    if out["cells"] is not None and li.cells_x > 0 and li.cells_y > 0:
        want_cells = oracle.cell_hist(want_bins, nb, d.scan.cell)
        assert np.array_equal(hog.level_cells(plan, out["cells"], l), want_cells), f"cells, level {l}"
    return want_bins


CASES = [
    dict(width=320, height=240, channels=1, n_bins=8),
    dict(width=800, height=600, channels=3, n_bins=9, norm=hog.HOG_NORM_L2),
    dict(width=333, height=277, channels=3, n_bins=18, max_levels=0, scale=1.2, norm=hog.HOG_NORM_L2),
    dict(width=130, height=131, channels=1, n_bins=64),
]


@pytest.mark.parametrize("bits", [16, 8])
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("from_planes", [False, True])
def test_narrow_planes_equal_oracle_mod_and_scores_equal_uint32(bits, case, from_planes):
    kw = CASES[case]
    img = inputs.synth_image(kw["width"], kw["height"], kw["channels"], 7100 + case)
    d32 = hog.make_desc(**kw)
    tmpl, bias = templates_for(d32, 7200 + case)
    plan32, out32 = run_gpu(d32, img, tmpl, bias, cell_hist=True, block_feat=False)
    plan, out = run_gpu(_desc(bits, **kw), img, tmpl, bias, cell_hist=True, block_feat=False,
                        cells_from_planes=from_planes)
    assert plan.sizes.ii_elem_bytes == bits // 8
    for l in range(plan.sizes.n_levels):
        li = plan.levels[l]
        assert li.ii_pitch * (bits // 8) % 128 == 0
        want_bins = _check_planes_and_cells(plan, out, img, l, bits)
        s = hog.level_scores(plan, out["scores"], l)
        s32 = hog.level_scores(plan32, out32["scores"], l)
        assert np.array_equal(s.view(np.uint32), s32.view(np.uint32)), f"scores, level {l}"
        if l == 0 and li.windows_x > 0:
            ref, absterm, _, wxs, wys = oracle.score_windows(want_bins, d32.n_bins, oracle_params(d32),
                                                             tmpl, bias)
            check_scores(s[wys, wxs, :], ref, absterm)


@pytest.mark.parametrize("bits,cell", [(8, 4), (8, 12), (8, 15), (16, 16), (16, 32), (16, 6)])
def test_other_cell_sizes_from_narrow_planes(bits, cell):
    """Cells other than 8 pixels are computed from the narrow planes: exact
    while cell^2 < 2^bits (15 x 15 = 225 < 256 is the largest for 8 bits)."""
    kw = dict(width=260, height=300, channels=3, n_bins=9, cell=cell, win_cells_x=4, win_cells_y=4,
              norm=hog.HOG_NORM_L2 if cell != 4 else hog.HOG_NORM_RAW)
    img = inputs.synth_image(260, 300, 3, 7300 + cell)
    tmpl, bias = templates_for(hog.make_desc(**kw), 7301 + cell)
    plan, out = run_gpu(_desc(bits, **kw), img, tmpl, bias, cell_hist=True, block_feat=False)
    want_bins = _check_planes_and_cells(plan, out, img, 0, bits)
    li = plan.levels[0]
    if li.windows_x:
        d = plan.desc
        ref, absterm, _, wxs, wys = oracle.score_windows(want_bins, d.n_bins, oracle_params(d), tmpl, bias)
        check_scores(hog.level_scores(plan, out["scores"], 0)[wys, wxs, :], ref, absterm)


@pytest.mark.parametrize("bits", [16, 8])
def test_wrapping_planes_on_a_full_hd_image(bits):
    """1920x1080: every count beyond 2^bits wraps, and the cells read from
    the wrapped planes are still exact."""
    kw = dict(width=1920, height=1080, channels=3, n_bins=8, norm=hog.HOG_NORM_L2)
    img = inputs.synth_image(1920, 1080, 3, 7400 + bits)
    tmpl, bias = templates_for(hog.make_desc(**kw), 7401)
    plan, out = run_gpu(_desc(bits, **kw), img, tmpl, bias, cell_hist=True, block_feat=False,
                        cells_from_planes=True)
    want_bins = _check_planes_and_cells(plan, out, img, 0, bits)
    full = oracle.integral(want_bins, 8)
    assert int(full.max()) >= 1 << 16  # the planes do wrap


@pytest.mark.parametrize("bits", [16, 8])
@pytest.mark.parametrize("nb,w,h", [(1, 70, 65), (5, 129, 66), (18, 257, 300), (64, 130, 131)])
def test_hog_integral_alone_on_random_bin_maps(bits, nb, w, h):
    import torch
    plan = hog.Plan(_desc(bits, width=w, height=h, channels=1, n_bins=nb))
    li = plan.levels[0]
    bm = inputs.synth_bin_map(w, h, nb, 7500 + nb)
    host = np.zeros(plan.sizes.bins_bytes, np.uint8)
    host[li.bins_offset: li.bins_offset + li.bins_pitch * h].reshape(h, li.bins_pitch)[:, :w] = bm
    buf = hog.Buffers(plan)
    buf.bins.copy_(torch.from_numpy(host))
    hog.hog_integral(plan, buf.bins, buf.ii, buf.workspace)
    torch.cuda.synchronize()
    got = hog.level_planes(plan, buf.ii.cpu().numpy(), 0)
    assert np.array_equal(got, oracle.integral_mod(bm, nb, bits)[:, 1:, 1:])


def test_batch_plan_with_8_bit_planes():
    sizes = [(320, 240), (201, 157), (640, 480), (64, 128)]
    descs = [_desc(8, width=w, height=h, channels=3, n_bins=8, max_levels=0, scale=1.3,
                   norm=hog.HOG_NORM_L2) for w, h in sizes]
    imgs = [inputs.synth_image(w, h, 3, 7600 + i) for i, (w, h) in enumerate(sizes)]
    tmpl, bias = templates_for(descs[0], 7601)
    plan, out = run_gpu_batch(descs, imgs, tmpl, bias)
    for i in range(len(sizes)):
        im = plan.images[i]
        for l in range(im.first_level, im.first_level + im.n_levels):
            _check_planes_and_cells(plan, out, imgs[i], l, 8, l0=im.first_level)
