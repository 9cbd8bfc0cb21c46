"""Scores within 1e-5 (sum_d |T_d f_d| + |b|) for templates whose weights span
any range of FP32 magnitudes, on both matrix-core scorers (the one-template
strip scorer, K < 16, and the window GEMM, K >= 16).

The templates are built against the image: ramps fill one known bin, and
huge weights sit on the bins the ramp never fills, so every score comes from
the small weights alone while each weight group's maximum is huge. The
strip scorer keeps weight ranges up to about 2^17 on its fp16 hi + lo split
and the window GEMM up to about 2^28 (its lo halves scaled by 2^11); wider
ranges (2^24 on the strips, 2^30, a single 2^40 outlier, 2^-60 weights beside
unit ones) take the exact FP32 path. Sec. 4 scores a window by the inner
product of its feature with the template; the oracle computes it in FP64.
"""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_params, run_gpu

pytestmark = pytest.mark.gpu

KINDS = ("huge_unfilled", "wide_split", "outlier", "tiny_filled")


def ramp(w, h, c, a, b, off=0):
    """P = a x + b y + off in every channel: every interior pixel has the same
    gradient (2a, 2b), so it lands in one bin."""
    y, x = np.mgrid[0:h, 0:w]
    p = a * x + b * y + off
    assert p.min() >= 0 and p.max() <= 255
    return np.repeat(p.astype(np.uint8)[:, :, None], c, axis=2)


def adversarial_templates(k, dim, nb, filled, seed, kinds):
    """k templates [k][dim] (FP32), template j of kind kinds[j % len(kinds)]:
    huge_unfilled  2^30 (random sign) on the bins the image never fills, N(0, 1) elsewhere
    wide_split     2^24 on the unfilled bins, |w| in [0.5, 1] elsewhere (the window
                   GEMM's scaled split; exact FP32 on the strips)
    outlier        N(0, 1) with one weight 2^40 on an unfilled bin
    tiny_filled    2^-60 N(0, 1) on the filled bins, N(0, 1) elsewhere"""
    rng = np.random.default_rng(seed)
    bins = np.arange(dim) % nb
    on = np.isin(bins, filled)
    out = np.empty((k, dim), np.float64)
    for j in range(k):
        kind = kinds[j % len(kinds)]
        sign = rng.choice([-1.0, 1.0], dim)
        g = rng.standard_normal(dim)
        if kind == "huge_unfilled":
            t = np.where(on, g, sign * 2.0 ** 30)
        elif kind == "wide_split":
            t = np.where(on, sign * rng.uniform(0.5, 1.0, dim), sign * 2.0 ** 24)
        elif kind == "outlier":
            t = g.copy()
            t[rng.choice(np.flatnonzero(~on))] = 2.0 ** 40
        elif kind == "tiny_filled":
            t = np.where(on, g * 2.0 ** -60, g)
        else:
            raise ValueError(kind)
        out[j] = t
    return out.astype(np.float32)


def check_all_levels(plan, out, img, tmpl, bias):
    d = plan.desc
    p = oracle_params(d)
    n = 0
    for l, li in enumerate(plan.levels):
        if li.windows_x == 0:
            continue
        lvl = img if l == 0 else oracle.resize_nn(img, li.scale, li.width, li.height)
        bins = oracle.bin_map(lvl, d.n_bins)
        s_ref, absterm, _, wxs, wys = oracle.score_windows(bins, d.n_bins, p, tmpl, bias)
        got = hog.level_scores(plan, out["scores"], l)[wys, wxs, :]
        check_scores(got, s_ref, absterm)
        n += got.size
    assert n > 0


def filled_bins(img, nb):
    b = oracle.bin_map(img, nb)
    return np.unique(b[b != oracle.NO_BIN])


# (n_bins, K, image (w, h, a, b), levels): K < 16 runs the strip scorer (8, 16
# and 20 bin slots per cell), K >= 16 the window GEMM (8 and 16 slots).
CASES = [
    (8, 1, (250, 200, 1, 0), 1),
    (8, 2, (100, 150, 1, 1), 1),
    (18, 1, (250, 200, 1, 0), 0),
    (18, 2, (250, 200, 1, 0), 1),
    (12, 1, (100, 150, 1, 1), 1),
    (8, 16, (250, 200, 1, 0), 1),
    (8, 32, (100, 150, 1, 1), 1),
    (16, 48, (250, 200, 1, 0), 0),
    (8, 48, (250, 200, 1, 0), 1),
]


@pytest.mark.parametrize("nb,k,geom,levels", CASES)
@pytest.mark.parametrize("kind", KINDS)
def test_matrix_scorers_adversarial_templates(nb, k, geom, levels, kind):
    w, h, a, b = geom
    desc = hog.make_desc(w, h, channels=3, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_L2,
                         max_levels=levels, scale=1.1)
    img = ramp(w, h, 3, a, b)
    fb = filled_bins(img, nb)
    assert len(fb) == 1
    dim = oracle_params(desc).dim(nb)
    tmpl = adversarial_templates(k, dim, nb, fb, 4242 + nb * 100 + k, (kind,))
    bias = np.zeros(k, np.float32)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    check_all_levels(plan, out, img, tmpl, bias)


@pytest.mark.parametrize("nb,k", [(8, 2), (18, 2), (8, 48), (16, 40)])
def test_matrix_scorers_mixed_templates_noise_image(nb, k):
    """Every kind in one call on a noise image (all bins filled): the kinds
    alternate across templates, so window-GEMM tiles mix split and exact
    templates, and the strip scorer picks the mode per template."""
    w, h = 300, 260
    desc = hog.make_desc(w, h, channels=3, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_L2)
    img = inputs.synth_image(w, h, 3, 4300 + nb + k)
    dim = oracle_params(desc).dim(nb)
    # "Unfilled" bins are the odd ones here: they do hold counts, so the huge
    # weights count in every score.
    tmpl = adversarial_templates(k, dim, nb, np.arange(0, nb, 2), 4400 + nb + k, KINDS)
    bias = np.linspace(-1.0, 1.0, k).astype(np.float32)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    check_all_levels(plan, out, img, tmpl, bias)


def test_window_gemm_split_and_exact_tiles():
    """K = 48: the first tile of 32 templates is within the split's range, the
    second holds 2^30-range templates; each tile scores in its own mode."""
    nb, k = 8, 48
    w, h = 250, 200
    desc = hog.make_desc(w, h, channels=3, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_L2)
    img = ramp(w, h, 3, 1, 0)
    fb = filled_bins(img, nb)
    dim = oracle_params(desc).dim(nb)
    t0 = adversarial_templates(32, dim, nb, fb, 4501, ("wide_split",))
    t1 = adversarial_templates(16, dim, nb, fb, 4502, ("huge_unfilled",))
    tmpl = np.concatenate([t0, t1])
    bias = np.zeros(k, np.float32)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    check_all_levels(plan, out, img, tmpl, bias)
