"""hog_run prepares the one-template strip scorer's weights inside the carry
scan's launch, four waves per template taking up to two block columns each;
the three separate calls (hog_integral, then hog_scan_windows) prepare them in
a launch of their own, one wave per block column. The two must give the same
fragments, so the same scores bit for bit: checked for 8, 16 and 20 bin slots
per cell (N_b 8, 16, 18), one and several templates, and templates in both
modes (fp16 hi + lo split and exact FP32), each also against the oracle (Sec. 4
inner product, FP64) within 1e-5 (sum |T f| + |b|)."""
import numpy as np
import pytest

from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import GuardedBuffers, oracle_params
from test_gpu_scorer_precision import adversarial_templates, check_all_levels, filled_bins, ramp

pytestmark = pytest.mark.gpu

# (n_bins, K, template kinds; None: N(0, 1) weights on a noise image)
CASES = [
    (8, 1, None),
    (16, 3, None),
    (18, 1, None),
    (18, 2, ("huge_unfilled", "wide_split")),
    (8, 3, ("tiny_filled", "outlier", "huge_unfilled")),
    (16, 1, ("wide_split",)),
]


def _run_both(desc, img, tmpl, bias):
    import torch
    plan = hog.Plan(desc)
    lut = hog.hog_lut_build(desc.n_bins)
    img_t = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda()
    tt = torch.from_numpy(np.ascontiguousarray(tmpl, np.float32).reshape(-1)).cuda()
    bt = torch.from_numpy(np.ascontiguousarray(bias, np.float32)).cuda()
    calls = GuardedBuffers(plan)
    fused = GuardedBuffers(plan)
    calls.scores.fill_(float("nan"))
    fused.scores.fill_(float("nan"))
    hog.run_path(plan, lut, img_t, tt, bt, calls)
    hog.hog_run(plan, lut, img_t, tt, bt, fused)
    torch.cuda.synchronize()
    return plan, calls.scores.cpu().numpy(), fused.scores.cpu().numpy()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_hog_run_fused_prep_equals_separate_prep(case):
    nb, k, kinds = CASES[case]
    w, h = 250, 200
    desc = hog.make_desc(w, h, channels=3, n_bins=nb, n_templates=k, norm=hog.HOG_NORM_L2,
                         max_levels=2, scale=1.1)
    dim = oracle_params(desc).dim(nb)
    if kinds is None:
        img = inputs.synth_image(w, h, 3, 4700 + case)
        tmpl = np.random.default_rng(4710 + case).standard_normal((k, dim)).astype(np.float32)
    else:
        img = ramp(w, h, 3, 1, 0)
        tmpl = adversarial_templates(k, dim, nb, filled_bins(img, nb), 4720 + case, kinds)
    bias = np.linspace(-0.5, 0.5, k).astype(np.float32)
    plan, s_calls, s_fused = _run_both(desc, img, tmpl, bias)
    n = plan.sizes.score_elems
    assert n > 0 and not np.isnan(s_fused[:n]).any()
    assert np.array_equal(s_calls[:n].view(np.uint32), s_fused[:n].view(np.uint32))
    check_all_levels(plan, dict(scores=s_fused), img, tmpl, bias)
