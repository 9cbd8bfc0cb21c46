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
    buf = GuardedBuffers(plan, cell_hist=cell_hist, block_feat=block_feat)
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
    buf = GuardedBuffers(plan, cell_hist=cell_hist, block_feat=l2)
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


# Canaries: every output buffer of a GPU test sits inside a larger allocation
# whose GUARD bytes before and after it hold a fixed pattern; after the test
# the pattern must be intact, so no kernel wrote outside the caller's buffers
# (the plane writer's duplicate stores into row padding and its buffer-range
# drops past a level's last row included).
GUARD = 64 * 1024
GUARD_BYTE = 0xA5
_guarded = []


class GuardedBuffers:
    """hog.Buffers with guard bands (same fields, same sizes)."""

    def __init__(self, plan, device="cuda", cell_hist=False, block_feat=False):
        import torch
        self._regions = []
        s = plan.sizes

        def alloc(name, n, dtype):
            esz = torch.empty(0, dtype=dtype).element_size()
            g = GUARD // esz
            base = torch.empty(n + 2 * g, dtype=dtype, device=device)
            base.view(torch.uint8).fill_(GUARD_BYTE)
            self._regions.append((name, base, g * esz, n * esz))
            return base[g:g + n]

        self.bins = alloc("bins", max(s.bins_bytes, 1), torch.uint8)
        self.ii = alloc("ii", max(s.ii_elems, 1), hog.ii_dtype(plan))
        self.scores = alloc("scores", max(s.score_elems, 1), torch.float32)
        self.workspace = alloc("workspace", max(s.workspace_bytes, 1), torch.uint8)
        self.cell_hist = alloc("cell_hist", max(s.cell_elems, 1), torch.int32) if cell_hist else None
        self.block_feat = alloc("block_feat", max(s.block_elems, 1), torch.float32) if block_feat else None
        _guarded.append(self)

    def check_guards(self):
        import torch
        for name, base, g, n in self._regions:
            b = base.view(torch.uint8)
            for part, view in (("before", b[:g]), ("after", b[g + n:])):
                bad = int((view != GUARD_BYTE).sum())
                assert bad == 0, f"{bad} bytes written {part} the {name} buffer"


def check_all_guards():
    """Check and forget every GuardedBuffers made since the last call."""
    import torch
    torch.cuda.synchronize()
    try:
        for b in _guarded:
            b.check_guards()
    finally:
        _guarded.clear()
