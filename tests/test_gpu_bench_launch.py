"""Every single-image benchmark workload at full size, launched as the
benchmark launches it: the plan, image and templates built by bench.py's own
workload_inputs, tiles autotuned on the same buffers, warm-up runs, then one
hog_run. Every level's bins and planes equal the oracle's bit for bit (mod
2^bits for narrow planes; weighted for soft votes); scores on sampled windows
of every level are within the stated tolerance."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog

from hog_cases import check_scores, oracle_params

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu

SINGLE = sorted(k for k, wl in bench.WORKLOADS.items() if "batch" not in wl)


def test_every_single_image_workload_is_covered():
    assert {"pyramid_1920x1080", "pyramid_1920x1080_u16", "pyramid_1920x1080_u8",
            "pyramid_1920x1080_soft", "rgb_800x600", "gray_320x240"} <= set(SINGLE)


@pytest.mark.parametrize("name", SINGLE)
def test_workload_in_the_benchmarked_launch_equals_oracle(name):
    import torch
    wl = bench.WORKLOADS[name]
    plan, imgs, host, tmpl, bias = bench.workload_inputs(wl)
    img = imgs[0]
    nb, bits = wl["n_bins"], wl.get("plane_bits", 32)
    soft = wl.get("votes", 0) == hog.HOG_VOTES_SOFT
    img_t = torch.from_numpy(host).cuda()
    tt, bt = torch.from_numpy(tmpl.reshape(-1)).cuda(), torch.from_numpy(bias).cuda()
    lut = hog.hog_lut_build(nb)
    buf = hog.Buffers(plan)
    stream = torch.cuda.current_stream()
    tiles = hog.autotune(plan, lut, img_t, tt, bt, buf, stream, reps=3)
    for _ in range(3):
        hog.hog_run(plan, lut, img_t, tt, bt, buf, stream)
    buf.scores.fill_(float("nan"))
    hog.hog_run(plan, lut, img_t, tt, bt, buf, stream)
    torch.cuda.synchronize()
    scores = buf.scores.cpu().numpy()
    bins_host = buf.bins.cpu().numpy()
    p = oracle_params(plan.desc)
    et = {4: np.uint32, 2: np.uint16, 1: np.uint8}[plan.sizes.ii_elem_bytes]
    rng = np.random.default_rng(77)
    for l in range(plan.sizes.n_levels):
        li = plan.levels[l]
        lvl = img if l == 0 else oracle.resize_nn(img, li.scale, li.width, li.height)
        what = f"{name} ({tiles}), level {l} ({li.width}x{li.height})"
        if soft:
            b0, w1 = oracle.soft_bin_map(lvl, nb, False)
            gb0, gw1 = hog.level_bins(plan, bins_host, l)
            assert np.array_equal(gb0, b0) and np.array_equal(gw1, w1), what
            want = oracle.soft_integral(b0, w1, nb)
        else:
            bins = oracle.bin_map(lvl, nb, False)
            assert np.array_equal(hog.level_bins(plan, bins_host, l), bins), what
            want = oracle.integral(bins, nb) if bits == 32 else oracle.integral_mod(bins, nb, bits)
        # Only this level's planes are copied back.
        n_el = li.ii_plane_stride * nb
        a = buf.ii.view(torch.uint8)[li.ii_offset * plan.sizes.ii_elem_bytes:
                                     (li.ii_offset + n_el) * plan.sizes.ii_elem_bytes].cpu().numpy().view(et)
        planes = a.reshape(nb, li.ii_plane_stride)[:, :li.ii_pitch * li.height]
        planes = planes.reshape(nb, li.height, li.ii_pitch)[:, :, :li.width]
        assert np.array_equal(planes, want[:, 1:, 1:]), what + " planes"
        if not li.windows_x:
            continue
        n = min(40, li.windows_x * li.windows_y)
        idx = rng.choice(li.windows_x * li.windows_y, size=n, replace=False)
        wxs, wys = idx % li.windows_x, idx // li.windows_x
        if soft:
            ref, absterm, wxs, wys = oracle.soft_score_windows(b0, w1, nb, p, tmpl, bias, wxs, wys)
        else:
            ref, absterm, _, wxs, wys = oracle.score_windows(bins, nb, p, tmpl, bias, wxs, wys)
        check_scores(hog.level_scores(plan, scores, l)[wys, wxs, :], ref, absterm)
    # Every score of the plan was written by the run.
    assert not np.isnan(scores[:plan.sizes.score_elems]).any(), name
