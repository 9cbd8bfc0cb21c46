"""Every weight position of the matrix-core scorers, one at a time.

A window's score is the inner product of its feature with the template
(Sec. 4); the feature concatenates the window's 2 x 2-cell blocks, 4 cells x
N_b bins each. Each template here is zero except the N_b bins of one cell of
one block position (by, bx), so its score is that one cell's contribution:
a weight fragment that is lost, misplaced or mixed with another step of the
products shows up as a wrong score. Every (by, bx, cell) position is covered,
for each bin-slot layout of the strip scorer (8, 16 and 20 slots per cell:
one, two, and two 32-feature steps plus a 16-feature step) and of the window
GEMM (8 and 16 slots), in the split fp16 mode and in the exact FP32 mode (a
2^-40 weight elsewhere in the template forces it; its product stays far below
the tolerance). The image is noise, so every bin of every cell holds counts.
"""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_params, run_gpu

pytestmark = pytest.mark.gpu

NBX, NBY = 7, 15  # block positions of a 64 x 128 window with 8-pixel cells


def position_templates(nb, positions, seed, exact):
    """One template per (by, bx, cell): N(0, 1) on that cell's bins, 0
    elsewhere (plus, when exact, a 2^-40 weight on the first bin of the same
    cell in the next block column)."""
    dim = NBX * NBY * 4 * nb
    rng = np.random.default_rng(seed)
    t = np.zeros((len(positions), dim), np.float32)
    for j, (by, bx, c) in enumerate(positions):
        base = ((by * NBX + bx) * 4 + c) * nb
        t[j, base:base + nb] = rng.standard_normal(nb).astype(np.float32)
        if exact:  # same block row (the strip scorer's scale group), next block column
            other = ((by * NBX + (bx + 1) % NBX) * 4 + c) * nb
            t[j, other] = np.float32(2.0 ** -40)
    return t


def run_positions(nb, positions, seed, exact, w=264, h=216):
    k = len(positions)
    desc = hog.make_desc(w, h, channels=3, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_L2)
    img = inputs.synth_image(w, h, 3, seed)
    tmpl = position_templates(nb, positions, seed + 1, exact)
    bias = np.zeros(k, np.float32)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    bins = oracle.bin_map(img, nb)
    s_ref, absterm, _, wxs, wys = oracle.score_windows(bins, nb, oracle_params(desc), tmpl, bias)
    got = hog.level_scores(plan, out["scores"], 0)[wys, wxs, :]
    check_scores(got, s_ref, absterm)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("nb", [8, 12, 18])
def test_strip_scorer_every_position(nb, exact):
    """K = 15 < 16 (strip scorer): template by covers block row by; one call
    per (bx, cell)."""
    for bx in range(NBX):
        for c in range(4):
            run_positions(nb, [(by, bx, c) for by in range(NBY)], 6100 + 10 * bx + c, exact)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("nb", [8, 16])
def test_window_gemm_every_position(nb, exact):
    """K = 32 (window GEMM): 420 positions in 14 calls of 32 templates."""
    allpos = [(by, bx, c) for by in range(NBY) for bx in range(NBX) for c in range(4)]
    for i in range(0, len(allpos), 32):
        run_positions(nb, allpos[i:i + 32], 6300 + i, exact)
