"""Level groups (hog_tiles.level_groups): hog_run splits a plan's levels into
contiguous ranges of about equal pixel counts and runs them on concurrent
streams, each range starting once the previous one writes its planes. Every
group count must give the one-group outputs bit for bit: single-image
pyramids and batch plans, every scorer, cells from the planes, narrow planes
and soft votes, inside a captured graph, and under concurrent calls on one
plan. The one-group outputs are tied to the oracle on sampled levels."""
import threading

import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_level_bins, oracle_params

pytestmark = pytest.mark.gpu

# (name, image sizes, make_desc keywords, templates)
CASES = [
    ("pyramid_strip_scorer", [(640, 480)], dict(channels=3, n_bins=18, max_levels=0, scale=1.05,
                                                norm=hog.HOG_NORM_L2), 1),
    ("batch_window_gemm", [(320, 240), (257, 301), (640, 360)],
     dict(channels=3, n_bins=8, max_levels=0, scale=1.1, norm=hog.HOG_NORM_L2), 32),
    ("gray_raw_vector_scorer", [(400, 300)], dict(channels=1, n_bins=9, max_levels=0, scale=1.1), 3),
    ("cells_from_planes", [(420, 330)], dict(channels=3, n_bins=8, max_levels=0, scale=1.1, cell=6,
                                             norm=hog.HOG_NORM_L2), 2),
    ("uint16_planes", [(500, 380)], dict(channels=3, n_bins=8, max_levels=0, scale=1.1,
                                         norm=hog.HOG_NORM_L2, plane_bits=16), 1),
    ("soft_votes", [(480, 360)], dict(channels=3, n_bins=9, max_levels=0, scale=1.1,
                                      norm=hog.HOG_NORM_L2, votes=hog.HOG_VOTES_SOFT), 1),
]


def _setup(sizes, kw, k, seed):
    import torch
    descs = [hog.make_desc(w, h, n_templates=k, **kw) for w, h in sizes]
    batch = len(sizes) > 1
    plan = hog.Plan(descs, batch=True) if batch else hog.Plan(descs[0])
    ch = kw.get("channels", 1)
    imgs = [inputs.synth_image(w, h, ch, seed + j) for j, (w, h) in enumerate(sizes)]
    host = hog.pack_images(plan, imgs) if batch else imgs[0].reshape(-1)
    img = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    tmpl, bias = inputs.synth_templates(k, plan.sizes.feature_dim, seed + 77)
    lut = hog.hog_lut_build(kw["n_bins"])
    return (plan, lut, imgs, img, tmpl, bias, torch.from_numpy(tmpl.reshape(-1)).cuda(),
            torch.from_numpy(bias).cuda())


def _snap(plan, buf):
    """Every defined output: all scores, each level's bins and planes."""
    import torch
    torch.cuda.synchronize()
    bins, ii = buf.bins.cpu().numpy(), buf.ii.cpu().numpy()
    out = [buf.scores.cpu().numpy().view(np.uint32)]
    for l in range(plan.sizes.n_levels):
        b = hog.level_bins(plan, bins, l)
        out += list(b) if isinstance(b, tuple) else [b]
        out.append(hog.level_planes(plan, ii, l))
    return out


@pytest.mark.parametrize("name,sizes,kw,k", CASES, ids=[c[0] for c in CASES])
def test_every_group_count_gives_the_one_group_outputs(name, sizes, kw, k):
    plan, lut, imgs, img, tmpl, bias, tt, bt = _setup(sizes, kw, k, 6100)
    t = hog.plan_tiles(plan)
    assert t.level_groups == 1  # plans start ungrouped
    buf = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    want = _snap(plan, buf)
    for g in range(2, hog.HOG_MAX_LEVEL_GROUPS + 1):
        hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, g)
        used = hog.plan_tiles(plan).level_groups
        assert 2 <= used <= g, (g, used)
        for rep in range(2):  # a repeated call reuses the plan's streams
            buf.scores.zero_()
            buf.ii.zero_()
            hog.hog_run(plan, lut, img, tt, bt, buf)
            for x, y in zip(want, _snap(plan, buf)):
                assert np.array_equal(x, y), (name, g, rep)
    # Back to one group.
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 0)
    assert hog.plan_tiles(plan).level_groups == 1
    hog.hog_run(plan, lut, img, tt, bt, buf)
    for x, y in zip(want, _snap(plan, buf)):
        assert np.array_equal(x, y)


def test_grouped_outputs_match_the_oracle_on_sampled_levels():
    """A 4-group pyramid against the oracle on its first, middle and last
    levels (one level from each end of the group ranges)."""
    plan, lut, imgs, img, tmpl, bias, tt, bt = _setup(*CASES[0][1:], 6200)
    t = hog.plan_tiles(plan)
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 4)
    buf = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    import torch
    torch.cuda.synchronize()
    bins, ii, scores = buf.bins.cpu().numpy(), buf.ii.cpu().numpy(), buf.scores.cpu().numpy()
    d = plan.desc
    p = oracle_params(d)
    L = plan.sizes.n_levels
    for l in sorted({0, L // 2, L - 1}):
        want = oracle_level_bins(imgs[0], plan, l)
        assert np.array_equal(hog.level_bins(plan, bins, l), want), l
        assert np.array_equal(hog.level_planes(plan, ii, l), oracle.integral(want, d.n_bins)[:, 1:, 1:]), l
        if plan.levels[l].windows_x:
            ref, absterm, _, _, _ = oracle.score_windows(want, d.n_bins, p, tmpl, bias)
            check_scores(hog.level_scores(plan, scores, l).reshape(ref.shape), ref, absterm)


@pytest.mark.parametrize("k", [1, 32])
def test_grouped_graph_replays_equal_eager(k):
    """A graph captured from a grouped plan (the groups' fork and join become
    graph edges): replays, with eager grouped runs between them, equal the
    one-group eager outputs bit for bit."""
    import torch
    kw = dict(channels=3, n_bins=8, max_levels=0, scale=1.1, norm=hog.HOG_NORM_L2)
    plan, lut, _, img, _, _, tt, bt = _setup([(320, 240), (257, 301), (640, 360)], kw, k, 6300)
    ref = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, ref)
    want = _snap(plan, ref)
    t = hog.plan_tiles(plan)
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 3)
    buf, other = hog.Buffers(plan), hog.Buffers(plan)
    g = hog.Graph(plan, lut, img, tt, bt, buf)
    for rep in range(3):
        g.launch()
        torch.cuda.synchronize()
        for x, y in zip(want, _snap(plan, buf)):
            assert np.array_equal(x, y), f"replay {rep}"
        hog.hog_run(plan, lut, img, tt, bt, other)  # eager grouped work between replays
        buf.scores.zero_()
        buf.ii.zero_()
        torch.cuda.synchronize()
    for x, y in zip(want, _snap(plan, other)):
        assert np.array_equal(x, y)
    g.destroy()


def test_concurrent_grouped_calls_on_one_plan():
    """Two host threads run one grouped plan on their own buffers and streams
    at the same time; each thread's outputs equal the one-group outputs."""
    import torch
    plan, lut, _, img, _, _, tt, bt = _setup(*CASES[0][1:], 6400)
    ref = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, ref)
    want = _snap(plan, ref)
    t = hog.plan_tiles(plan)
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 2)
    bufs = [hog.Buffers(plan), hog.Buffers(plan)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    errors = []

    def worker(i):
        try:
            torch.cuda.set_device(0)
            for _ in range(20):
                hog.hog_run(plan, lut, img, tt, bt, bufs[i], streams[i])
            streams[i].synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errors, errors
    for b in bufs:
        for x, y in zip(want, _snap(plan, b)):
            assert np.array_equal(x, y)


def test_autotune_chooses_a_group_count():
    plan, lut, _, img, _, _, tt, bt = _setup(*CASES[1][1:], 6500)
    buf = hog.Buffers(plan)
    hog.hog_run(plan, lut, img, tt, bt, buf)
    want = _snap(plan, buf)
    t = hog.autotune(plan, lut, img, tt, bt, buf, reps=2)
    assert 1 <= t.level_groups <= hog.HOG_MAX_LEVEL_GROUPS
    assert hog.plan_tiles(plan).level_groups == t.level_groups
    buf.scores.zero_()
    hog.hog_run(plan, lut, img, tt, bt, buf)
    for x, y in zip(want, _snap(plan, buf)):
        assert np.array_equal(x, y)


def test_bad_group_counts_are_rejected_and_single_levels_stay_ungrouped():
    kw = dict(channels=1, n_bins=8)
    plan, *_ = _setup([(200, 150)], kw, 1, 6600)  # one level
    t = hog.plan_tiles(plan)
    for g in (-1, hog.HOG_MAX_LEVEL_GROUPS + 1):
        with pytest.raises(hog.HogError) as e:
            hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, g)
        assert e.value.status == hog.HOG_E_INVALID
    hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 4)
    assert hog.plan_tiles(plan).level_groups == 1
