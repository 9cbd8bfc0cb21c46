"""Batch plans: several images of different sizes, each with its own pyramid,
in one launch per kernel. Every level of every image is compared with the
oracle, and each image's results must equal, bit for bit, those of a
single-image plan of the same image (alone and in the mix give the same
result)."""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import (check_scores, oracle_level_bins, oracle_params, run_gpu, run_gpu_batch,
                       templates_for)

pytestmark = pytest.mark.gpu


def _check_image(plan, out, img, i, tmpl, bias):
    info = plan.images[i]
    d = plan.descs[i]
    nb = d.n_bins
    p = oracle_params(d)
    for l in range(info.first_level, info.first_level + info.n_levels):
        li = plan.levels[l]
        want = oracle_level_bins(img, plan, l, info.first_level)
        assert np.array_equal(hog.level_bins(plan, out["bins"], l), want), f"image {i} level {l} bins"
        assert np.array_equal(hog.level_planes(plan, out["ii"], l),
                              oracle.integral(want, nb)[:, 1:, 1:]), f"image {i} level {l} planes"
        if li.cells_x and li.cells_y:
            assert np.array_equal(hog.level_cells(plan, out["cells"], l),
                                  oracle.cell_hist(want, nb, d.scan.cell)), f"image {i} level {l} cells"
        if li.windows_x:
            ref, absterm, _, _, _ = oracle.score_windows(want, nb, p, tmpl, bias)
            got = hog.level_scores(plan, out["scores"], l).reshape(ref.shape)
            check_scores(got, ref, absterm)


def _same_as_alone(plan, out, imgs, tmpl, bias):
    """Each image alone (single-image plan) gives bit-identical outputs."""
    for i, img in enumerate(imgs):
        info = plan.images[i]
        p1, o1 = run_gpu(plan.descs[i], img, tmpl, bias)
        assert p1.sizes.n_levels == info.n_levels
        for k in range(info.n_levels):
            l = info.first_level + k
            assert np.array_equal(hog.level_bins(plan, out["bins"], l), hog.level_bins(p1, o1["bins"], k))
            assert np.array_equal(hog.level_planes(plan, out["ii"], l), hog.level_planes(p1, o1["ii"], k))
            a = hog.level_scores(plan, out["scores"], l)
            b = hog.level_scores(p1, o1["scores"], k)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"image {i} level {k} scores"


RGB_SIZES = [(230, 300), (65, 129), (320, 240), (401, 183), (64, 128), (60, 100), (129, 257)]


def test_rgb_l2_pyramid_batch():
    """RGB, N_b = 8, 1.1 pyramids, 2x2-cell L2 blocks, two templates; one image
    smaller than a window."""
    descs = [hog.make_desc(w, h, channels=3, n_bins=8, max_levels=0, scale=1.1, n_templates=2,
                           norm=hog.HOG_NORM_L2) for w, h in RGB_SIZES]
    imgs = [inputs.synth_image(w, h, 3, inputs.SEED_BATCH_BASE + j) for j, (w, h) in enumerate(RGB_SIZES)]
    tmpl, _ = templates_for(descs[0], 4100)
    bias = np.array([0.25, -1.5], np.float32)
    plan, out = run_gpu_batch(descs, imgs, tmpl, bias)
    assert len(plan.images) == len(RGB_SIZES)
    assert plan.sizes.n_levels == sum(im.n_levels for im in plan.images)
    for i, img in enumerate(imgs):
        _check_image(plan, out, img, i, tmpl, bias)
    _same_as_alone(plan, out, imgs, tmpl, bias)


def test_gray_raw_batch_single_levels():
    sizes = [(320, 240), (70, 130), (200, 150), (3, 3)]
    descs = [hog.make_desc(w, h, channels=1, n_bins=9) for w, h in sizes]
    imgs = [inputs.synth_image(w, h, 1, 4200 + j) for j, (w, h) in enumerate(sizes)]
    tmpl, bias = templates_for(descs[0], 4300)
    plan, out = run_gpu_batch(descs, imgs, tmpl, bias)
    for i, img in enumerate(imgs):
        _check_image(plan, out, img[:, :, 0], i, tmpl, bias)
    _same_as_alone(plan, out, [im[:, :, 0] for im in imgs], tmpl, bias)


def test_batch_n18_mixed_pyramids():
    """N_b = 18 (three 6-bin chunks), images with and without pyramids."""
    sizes = [(300, 260, 0), (257, 140, 1), (150, 300, 3)]
    descs = [hog.make_desc(w, h, channels=3, n_bins=18, max_levels=ml, scale=1.05,
                           norm=hog.HOG_NORM_L2) for w, h, ml in sizes]
    imgs = [inputs.synth_image(w, h, 3, 4400 + j) for j, (w, h, _) in enumerate(sizes)]
    tmpl, bias = templates_for(descs[0], 4500)
    plan, out = run_gpu_batch(descs, imgs, tmpl, bias)
    for i, img in enumerate(imgs):
        _check_image(plan, out, img, i, tmpl, bias)


def _batch_setup(sizes, k, seed):
    import torch
    descs = [hog.make_desc(w, h, channels=3, n_bins=8, max_levels=0, scale=1.1, n_templates=k,
                           norm=hog.HOG_NORM_L2) for w, h in sizes]
    plan = hog.Plan(descs, batch=True)
    lut = hog.hog_lut_build(8)
    imgs = [inputs.synth_image(w, h, 3, seed + j) for j, (w, h) in enumerate(sizes)]
    packed = torch.from_numpy(hog.pack_images(plan, imgs)).cuda()
    tmpl, bias = inputs.synth_templates(k, plan.sizes.feature_dim, seed + 99)
    return (plan, lut, imgs, packed, torch.from_numpy(tmpl.reshape(-1)).cuda(),
            torch.from_numpy(bias).cuda())


def _snap(plan, buf):
    """The defined part of every output: each level's bins and planes (row
    padding is unspecified) and all scores."""
    bins, ii = buf.bins.cpu().numpy(), buf.ii.cpu().numpy()
    out = [buf.scores.cpu().numpy().view(np.uint32)]
    for l in range(plan.sizes.n_levels):
        out.append(hog.level_bins(plan, bins, l))
        out.append(hog.level_planes(plan, ii, l))
    return out


def test_hog_run_equals_the_three_calls():
    import torch
    plan, lut, _, packed, tt, bt = _batch_setup([(300, 200), (130, 257)], 2, 4600)
    b1, b2 = hog.Buffers(plan), hog.Buffers(plan)
    hog.run_path(plan, lut, packed, tt, bt, b1)
    hog.hog_run(plan, lut, packed, tt, bt, b2)
    torch.cuda.synchronize()
    for x, y in zip(_snap(plan, b1), _snap(plan, b2)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("k", [1, 32])
def test_graph_replays_equal_eager(k):
    """hog_graph: replays with eager work between them, and after the input
    is refilled in place, give the eager results bit for bit."""
    import torch
    sizes = [(320, 240), (257, 301), (640, 360)]
    plan, lut, imgs, packed, tt, bt = _batch_setup(sizes, k, 4700)
    ref = hog.Buffers(plan)
    hog.hog_run(plan, lut, packed, tt, bt, ref)
    torch.cuda.synchronize()
    want = _snap(plan, ref)
    buf = hog.Buffers(plan)
    g = hog.Graph(plan, lut, packed, tt, bt, buf)
    other = hog.Buffers(plan)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for x, y in zip(want, _snap(plan, buf)):
            assert np.array_equal(x, y), f"replay {rep}"
        hog.hog_run(plan, lut, packed, tt, bt, other)  # eager work between replays
        buf.scores.zero_()
        torch.cuda.synchronize()
    # New image contents in the same buffer: the replay reads them.
    imgs2 = [inputs.synth_image(w, h, 3, 4800 + j) for j, (w, h) in enumerate(sizes)]
    packed.copy_(torch.from_numpy(hog.pack_images(plan, imgs2)))
    g.launch()
    hog.hog_run(plan, lut, packed, tt, bt, other)
    torch.cuda.synchronize()
    for x, y in zip(_snap(plan, other), _snap(plan, buf)):
        assert np.array_equal(x, y)
    g.destroy()


def test_full_batch64_in_the_benchmarked_launch():
    """The batched workload at full size, launched as the benchmark launches
    it: 64 RGB images of seeded uniform sizes in 320..1920 x 240..1080 with
    1.1 pyramids (1,088 levels), N_b = 8, L2, K = 32, tiles autotuned, one
    captured graph replayed. Sampled images and levels: bins, planes and
    cells bit for bit; scores on sampled windows within tolerance. Only the
    checked levels are copied back."""
    import os
    import sys
    import torch
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    wl = bench.WORKLOADS["batch64"]
    plan, imgs, host, tmpl, bias = bench.workload_inputs(wl)
    descs = plan.descs
    assert plan.sizes.n_levels == 1088 and tmpl.shape[0] == 32
    packed = torch.from_numpy(host).cuda()
    tt, bt = torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda()
    lut = hog.hog_lut_build(8)
    buf = hog.Buffers(plan, cell_hist=False, block_feat=False)
    hog.autotune(plan, lut, packed, tt, bt, buf)
    buf.scores.zero_()
    g = hog.Graph(plan, lut, packed, tt, bt, buf)
    g.launch()
    torch.cuda.synchronize()
    scores = buf.scores.cpu().numpy()
    p = oracle_params(descs[0])
    rng = np.random.default_rng(64)
    for i in sorted(rng.choice(64, size=4, replace=False)):
        info = plan.images[i]
        ls = sorted({info.first_level, info.first_level + info.n_levels // 2,
                     info.first_level + info.n_levels - 1})
        for l in ls:
            li = plan.levels[l]
            want = oracle_level_bins(imgs[i], plan, l, info.first_level)
            bins = buf.bins[li.bins_offset: li.bins_offset + li.bins_pitch * li.height].cpu().numpy()
            assert np.array_equal(bins.reshape(li.height, li.bins_pitch)[:, :li.width], want), f"image {i} level {l}"
            ii = buf.ii[li.ii_offset: li.ii_offset + li.ii_plane_stride * 8].cpu().numpy().view(np.uint32)
            planes = ii.reshape(8, li.ii_plane_stride)[:, :li.ii_pitch * li.height]
            planes = planes.reshape(8, li.height, li.ii_pitch)[:, :, :li.width]
            assert np.array_equal(planes, oracle.integral(want, 8)[:, 1:, 1:]), f"image {i} level {l} planes"
            if li.windows_x:
                n = min(40, li.windows_x * li.windows_y)
                idx = rng.choice(li.windows_x * li.windows_y, size=n, replace=False)
                ref, absterm, _, wxs, wys = oracle.score_windows(want, 8, p, tmpl, bias, idx % li.windows_x,
                                                                 idx // li.windows_x)
                check_scores(hog.level_scores(plan, scores, l)[wys, wxs, :], ref, absterm)
    g.destroy()


@pytest.mark.parametrize("variant", [dict(plane_bits=8), dict(plane_bits=16), dict(votes=1)])
def test_variants_in_batch_plans_graphs_and_autotune(variant):
    """Narrow planes and soft votes through a batch plan, the autotuner and a
    captured graph: the graph's replays equal an eager hog_run bit for bit,
    and each image's scores equal its single-image plan's."""
    import torch
    sizes = [(320, 240), (257, 301), (96, 160)]
    descs = [hog.make_desc(w, h, channels=3, n_bins=8, max_levels=0, scale=1.2, n_templates=2,
                           norm=hog.HOG_NORM_L2, **variant) for w, h in sizes]
    plan = hog.Plan(descs, batch=True)
    lut = hog.hog_lut_build(8)
    imgs = [inputs.synth_image(w, h, 3, 4900 + j) for j, (w, h) in enumerate(sizes)]
    packed = torch.from_numpy(hog.pack_images(plan, imgs)).cuda()
    tmpl, bias = inputs.synth_templates(2, plan.sizes.feature_dim, 4999)
    tt, bt = torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda()
    ref = hog.Buffers(plan)
    hog.autotune(plan, lut, packed, tt, bt, ref)
    hog.hog_run(plan, lut, packed, tt, bt, ref)
    torch.cuda.synchronize()
    want = _snap(plan, ref)
    buf = hog.Buffers(plan)
    g = hog.Graph(plan, lut, packed, tt, bt, buf)
    for rep in range(2):
        g.launch()
        torch.cuda.synchronize()
        for x, y in zip(want, _snap(plan, buf)):
            assert np.array_equal(x, y), f"replay {rep}"
        buf.scores.zero_()
    g.destroy()
    scores = ref.scores.cpu().numpy()
    for i, img in enumerate(imgs):
        info = plan.images[i]
        p1, o1 = run_gpu(descs[i], img, tmpl, bias, cell_hist=False, block_feat=False)
        for k in range(info.n_levels):
            a = hog.level_scores(plan, scores, info.first_level + k)
            b = hog.level_scores(p1, o1["scores"], k)
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"image {i} level {k}"
