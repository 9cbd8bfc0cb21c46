"""Shared helpers for the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

# Tolerance stated for FP32 features and scores: 1e-5 relative; for scores the
# scale is sum_d |T_d f_d| + |b| (a score near 0 has no relative meaning).
FEAT_RTOL = 1e-5
SCORE_RTOL = 1e-5


def run_gpu(desc: hog.PlanDesc, img: np.ndarray, tmpl: np.ndarray, bias: np.ndarray,
            cell_hist=True, block_feat=None, repeat=1, cells_from_planes=False,
            orientation=hog.HOG_ORIENT_SIGNED):
    """Run the three calls on cuda:0; return host copies of every output."""
    import torch
    plan = hog.Plan(desc)
    lut = hog.hog_lut_build(desc.n_bins, orientation)
    if block_feat is None:
        block_feat = desc.scan.norm == hog.HOG_NORM_L2
    buf = hog.Buffers(plan, cell_hist=cell_hist, block_feat=block_feat)
    img_t = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).to("cuda")
    tmpl_t = torch.from_numpy(np.ascontiguousarray(tmpl, np.float32).reshape(-1)).to("cuda")
    bias_t = torch.from_numpy(np.ascontiguousarray(bias, np.float32).reshape(-1)).to("cuda")
    outs = []
    for _ in range(repeat):
        hog.run_path(plan, lut, img_t, tmpl_t, bias_t, buf, cells_from_planes=cells_from_planes)
        torch.cuda.synchronize()
        outs.append(dict(
            bins=buf.bins.cpu().numpy(),
            ii=buf.ii.cpu().numpy(),
            scores=buf.scores.cpu().numpy(),
            cells=buf.cell_hist.cpu().numpy() if buf.cell_hist is not None else None,
            blocks=buf.block_feat.cpu().numpy() if buf.block_feat is not None else None,
        ))
    return plan, (outs[0] if repeat == 1 else outs)


def oracle_level_bins(img: np.ndarray, plan: hog.Plan, l: int, l0: int = 0,
                      unsigned: bool = False) -> np.ndarray:
    """Oracle bins of plan level l, which belongs to the image whose first
    level is l0 (0 for single-image plans)."""
    li = plan.levels[l]
    nb = plan.desc.n_bins
    if l == l0:
        return oracle.bin_map(img, nb, unsigned)
    lvl = oracle.resize_nn(img, li.scale, li.width, li.height)
    return oracle.bin_map(lvl, nb, unsigned)


def run_gpu_batch(descs, imgs, tmpl: np.ndarray, bias: np.ndarray, cell_hist=True):
    """Run the three calls on one batch plan over imgs (packed as the plan
    says); return the plan and host copies of every output."""
    import torch
    plan = hog.Plan(descs, batch=True)
    lut = hog.hog_lut_build(plan.desc.n_bins)
    l2 = plan.desc.scan.norm == hog.HOG_NORM_L2
    buf = hog.Buffers(plan, cell_hist=cell_hist, block_feat=l2)
    packed = torch.from_numpy(hog.pack_images(plan, imgs)).to("cuda")
    tmpl_t = torch.from_numpy(np.ascontiguousarray(tmpl, np.float32).reshape(-1)).to("cuda")
    bias_t = torch.from_numpy(np.ascontiguousarray(bias, np.float32).reshape(-1)).to("cuda")
    hog.run_path(plan, lut, packed, tmpl_t, bias_t, buf)
    torch.cuda.synchronize()
    return plan, dict(bins=buf.bins.cpu().numpy(), ii=buf.ii.cpu().numpy(),
                      scores=buf.scores.cpu().numpy(),
                      cells=buf.cell_hist.cpu().numpy() if buf.cell_hist is not None else None,
                      blocks=buf.block_feat.cpu().numpy() if buf.block_feat is not None else None)


def oracle_params(desc: hog.PlanDesc) -> oracle.ScanParams:
    s = desc.scan
    return oracle.ScanParams(cell=s.cell, win_cells_x=s.win_cells_x, win_cells_y=s.win_cells_y,
                             block=s.block, norm=s.norm, eps=1e-3 if s.eps == 0 else float(s.eps))


def check_scores(got: np.ndarray, ref: np.ndarray, absterm: np.ndarray):
    err = np.abs(got.astype(np.float64) - ref)
    bound = SCORE_RTOL * absterm
    bad = err > bound
    assert not bad.any(), (
        f"{bad.sum()} scores out of tolerance; worst err/bound "
        f"{np.max(err / np.maximum(bound, 1e-300)):.3g}")


def check_features(got: np.ndarray, ref: np.ndarray):
    zero = ref == 0
    assert np.all(got[zero] == 0), "empty block must give exact zeros"
    err = np.abs(got.astype(np.float64) - ref)
    bad = (err > FEAT_RTOL * np.abs(ref)) & ~zero
    assert not bad.any(), f"{bad.sum()} features out of tolerance; worst rel err " \
                          f"{np.max(err[~zero] / np.abs(ref[~zero])):.3g}"


def templates_for(desc: hog.PlanDesc, seed: int):
    plan_dim = oracle_params(desc).dim(desc.n_bins)
    return inputs.synth_templates(desc.n_templates, plan_dim, seed)
