"""A seeded sweep over combinations of the variants that other tests fix one
at a time: image size and channels, bin count, orientation, hard or soft
votes, plane width, cell size, normalisation, template count (and so the
scorer) and pyramid. Every level's bins, planes and cells equal the
oracle's bit for bit; scores are within the stated tolerance on sampled
windows."""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_params, run_gpu, templates_for

pytestmark = pytest.mark.gpu


def _configs(n=48, seed=8100):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        votes = int(rng.random() < 0.3)
        bits = 32 if votes else int(rng.choice([32, 32, 16, 8]))
        cell = int(rng.choice([8, 8, 4, 6, 12]))
        if cell * cell >= (1 << bits):  # the plan requires cell^2 < 2^bits
            continue
        multi = bool(rng.random() < 0.5)
        out.append(dict(width=int(rng.integers(3, 700)), height=int(rng.integers(3, 520)),
                        channels=int(rng.choice([1, 3])),
                        n_bins=int(rng.choice([1, 2, 3, 8, 9, 13, 18, 36, 64])),
                        n_templates=int(rng.choice([1, 1, 2, 5, 16, 32])), cell=cell,
                        norm=int(rng.integers(0, 2)), plane_bits=bits, votes=votes,
                        max_levels=0 if multi else 1, scale=float(rng.choice([1.1, 1.3])),
                        orientation=int(rng.integers(0, 2))))
    return out


CONFIGS = _configs()


@pytest.mark.parametrize("i", range(len(CONFIGS)))
def test_random_config_equals_oracle(i):
    c = dict(CONFIGS[i])
    orientation = c.pop("orientation")
    unsigned = orientation == hog.HOG_ORIENT_UNSIGNED
    desc = hog.make_desc(**c)
    img = inputs.synth_image(c["width"], c["height"], c["channels"], 8200 + i)
    tmpl, bias = templates_for(desc, 8300 + i)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=True, block_feat=False, orientation=orientation)
    nb, cell, bits = c["n_bins"], c["cell"], c["plane_bits"]
    p = oracle_params(desc)
    rng = np.random.default_rng(8400 + i)
    for l in range(plan.sizes.n_levels):
        li = plan.levels[l]
        lvl = img if l == 0 else oracle.resize_nn(img, li.scale, li.width, li.height)
        what = f"config {i} {CONFIGS[i]}, level {l} ({li.width}x{li.height})"
        if c["votes"]:
            b0, w1 = oracle.soft_bin_map(lvl, nb, unsigned)
            gb0, gw1 = hog.level_bins(plan, out["bins"], l)
            assert np.array_equal(gb0, b0) and np.array_equal(gw1, w1), what
            planes = oracle.soft_integral(b0, w1, nb)
            cells = oracle.soft_cell_hist(b0, w1, nb, cell)
        else:
            bins = oracle.bin_map(lvl, nb, unsigned)
            assert np.array_equal(hog.level_bins(plan, out["bins"], l), bins), what
            planes = oracle.integral(bins, nb) if bits == 32 else oracle.integral_mod(bins, nb, bits)
            cells = oracle.cell_hist(bins, nb, cell)
        assert np.array_equal(hog.level_planes(plan, out["ii"], l), planes[:, 1:, 1:]), what
        if li.cells_x and li.cells_y:
            assert np.array_equal(hog.level_cells(plan, out["cells"], l), cells), what
        if not li.windows_x:
            continue
        n = min(40, li.windows_x * li.windows_y)
        idx = rng.choice(li.windows_x * li.windows_y, size=n, replace=False)
        wxs, wys = idx % li.windows_x, idx // li.windows_x
        if c["votes"]:
            ref, absterm, wxs, wys = oracle.soft_score_windows(b0, w1, nb, p, tmpl, bias, wxs, wys)
        else:
            ref, absterm, _, wxs, wys = oracle.score_windows(bins, nb, p, tmpl, bias, wxs, wys)
        check_scores(hog.level_scores(plan, out["scores"], l)[wys, wxs, :], ref, absterm)


def _batches(n=8, seed=8500):
    rng = np.random.default_rng(seed)
    out = []
    for c in _configs(n, seed):
        k = int(rng.integers(2, 7))
        sizes = [(int(rng.integers(3, 500)), int(rng.integers(3, 400))) for _ in range(k)]
        out.append((c, sizes, int(rng.integers(1, hog.HOG_MAX_LEVEL_GROUPS + 1))))
    return out


BATCHES = _batches()


@pytest.mark.parametrize("i", range(len(BATCHES)))
def test_random_batch_with_level_groups_equals_oracle(i):
    """Batch plans of uneven images sharing a random variant setting, run by
    hog_run with a random number of level groups: each image's levels equal
    the oracle (bins, planes bit for bit; sampled scores within tolerance)."""
    import torch
    c, sizes, groups = BATCHES[i]
    c = dict(c)
    orientation = c.pop("orientation")
    unsigned = orientation == hog.HOG_ORIENT_UNSIGNED
    descs = [hog.make_desc(**dict(c, width=w, height=h)) for w, h in sizes]
    plan = hog.Plan(descs, batch=True)
    imgs = [inputs.synth_image(w, h, c["channels"], 8600 + 10 * i + j) for j, (w, h) in enumerate(sizes)]
    tmpl, bias = templates_for(descs[0], 8700 + i)
    lut = hog.hog_lut_build(c["n_bins"], orientation)
    t = hog.plan_tiles(plan)
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, groups)
    buf = hog.Buffers(plan)
    packed = torch.from_numpy(hog.pack_images(plan, imgs)).cuda()
    hog.hog_run(plan, lut, packed, torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda(), buf)
    torch.cuda.synchronize()
    out_bins, out_ii, out_scores = buf.bins.cpu().numpy(), buf.ii.cpu().numpy(), buf.scores.cpu().numpy()
    nb, bits = c["n_bins"], c["plane_bits"]
    p = oracle_params(descs[0])
    rng = np.random.default_rng(8800 + i)
    for j, img in enumerate(imgs):
        info = plan.images[j]
        for k in range(info.n_levels):
            l = info.first_level + k
            li = plan.levels[l]
            lvl = img if k == 0 else oracle.resize_nn(img, li.scale, li.width, li.height)
            what = f"batch {i} {BATCHES[i]}, image {j}, level {k} ({li.width}x{li.height})"
            if c["votes"]:
                b0, w1 = oracle.soft_bin_map(lvl, nb, unsigned)
                gb0, gw1 = hog.level_bins(plan, out_bins, l)
                assert np.array_equal(gb0, b0) and np.array_equal(gw1, w1), what
                planes = oracle.soft_integral(b0, w1, nb)
            else:
                bins = oracle.bin_map(lvl, nb, unsigned)
                assert np.array_equal(hog.level_bins(plan, out_bins, l), bins), what
                planes = oracle.integral(bins, nb) if bits == 32 else oracle.integral_mod(bins, nb, bits)
            assert np.array_equal(hog.level_planes(plan, out_ii, l), planes[:, 1:, 1:]), what
            if not li.windows_x:
                continue
            n = min(20, li.windows_x * li.windows_y)
            idx = rng.choice(li.windows_x * li.windows_y, size=n, replace=False)
            wxs, wys = idx % li.windows_x, idx // li.windows_x
            if c["votes"]:
                ref, absterm, wxs, wys = oracle.soft_score_windows(b0, w1, nb, p, tmpl, bias, wxs, wys)
            else:
                ref, absterm, _, wxs, wys = oracle.score_windows(bins, nb, p, tmpl, bias, wxs, wys)
            check_scores(hog.level_scores(plan, out_scores, l)[wys, wxs, :], ref, absterm)
