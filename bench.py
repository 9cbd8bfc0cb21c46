"""Benchmark of the fast-HOG hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole path over one synthetic image: one hog_run
(bin map of every pyramid level, one integral image per bin per level, cells,
blocks and window scores) through the C ABI, with the image, templates and
all buffers resident in HBM. With
--workload batch64 a step is one pass over a batch of 64 images (one batch
plan, replayed as a captured HIP graph); the line then also gives the same
images run through 64 single-image plans, one after another. With
--workload serve [--rate R] [--requests N] a Poisson stream of mixed-size
requests goes through the request server (hog_submit / hog_wait_any /
hog_poll) and, for comparison, through the per-image path; the value is the
server's throughput at that offered load, with its latency percentiles.

Prints one JSON line: processed Mpixel/s (pixels summed over pyramid
levels), per-step latency percentiles (at least 200 single-step samples),
per-kernel times, the roofline of the dominant kernel (the integral-image
writer) measured live with HIP events (beside this GPU's own 1 GiB copy and
fill rates) and of the whole path (its algorithmic bytes per step over the
step time), the rate with the image copied from pinned host memory each
step, the input's bin statistics, and the CPU oracle timed on this host
over one full step, single-threaded and split by level across the host's
cores. Steps cycle through distinct buffer sets totalling at least
--ring-bytes (1 GiB), so that a small workload is timed from HBM and not
from the last-level cache; the two small workloads also report their
batched form (one batch plan of many such images, one graph launch).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
H2D_PASSES = 3  # timed passes behind each host-to-device copy figure
METRIC = "Mpixel/s end-to-end (bins+integrals+window scores) vs HBM roofline; p99 latency"

WORKLOADS = {
    # 1920x1080 RGB, N_b = 18, nearest-neighbour pyramid at 1.05 down to the
    # 64x128 window (44 levels), 2x2-cell L2 blocks (7560-dim), one template.
    "pyramid_1920x1080": dict(width=1920, height=1080, channels=3, n_bins=18, max_levels=0,
                              scale=1.05, norm=1, seed=1002, tseed=9002),
    # 800x600 RGB, N_b = 8, single level, L2 blocks (3360-dim), one template.
    "rgb_800x600": dict(width=800, height=600, channels=3, n_bins=8, max_levels=1, scale=1.0,
                        norm=1, seed=1001, tseed=9001, batched_form=64, oracle_images=16),
    # 320x240 grey, N_b = 8, single level, raw 8x16x8 cell features.
    "gray_320x240": dict(width=320, height=240, channels=1, n_bins=8, max_levels=1, scale=1.0,
                         norm=0, seed=1000, tseed=9000, batched_form=400, oracle_images=192),
    # Batched: 64 RGB images, sizes uniform in 320..1920 x 240..1080 (seeded),
    # each with a 1.1 pyramid, N_b = 8, L2 blocks (3360-dim), 32 templates; one
    # batch plan replayed as a captured HIP graph, beside the same 64 images
    # run through 64 single-image plans.
    "batch64": dict(batch=64, size_seed=4000, channels=3, n_bins=8, max_levels=0, scale=1.1,
                    norm=1, seed=4000, tseed=9003, templates=32),
    # The pyramid workload with narrow integral images: uint16 / uint8 planes
    # holding the counts mod 2^16 / 2^8 (exact four-corner sums for areas
    # below 2^16 / 2^8 pixels; the 8x8 cells and the scores are unchanged).
    "pyramid_1920x1080_u16": dict(width=1920, height=1080, channels=3, n_bins=18, max_levels=0,
                                  scale=1.05, norm=1, seed=1002, tseed=9002, plane_bits=16),
    "pyramid_1920x1080_u8": dict(width=1920, height=1080, channels=3, n_bins=18, max_levels=0,
                                 scale=1.05, norm=1, seed=1002, tseed=9002, plane_bits=8),
    # The pyramid workload with two-bin soft votes (quantised to 1/32 pixel):
    # weighted uint32 planes, each written once (tile reduce, prefixes, writer).
    "pyramid_1920x1080_soft": dict(width=1920, height=1080, channels=3, n_bins=18, max_levels=0,
                                   scale=1.05, norm=1, seed=1002, tseed=9002, votes=1),
}
KERNELS = ("bin_map", "integral_reduce", "integral_scan", "integral_emit", "integral_soft", "cells", "score")


def kernel_sources_sha256():
    h = hashlib.sha256()
    for f in ("hog_kernels.hip", "hog_internal.h"):
        with open(os.path.join(ROOT, "paper_1703_06256_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, bin_chunk):
    """HBM bytes per integral_emit launch with `bin_chunk` bins per wave from
    the committed FETCH_SIZE / WRITE_SIZE summary of this workload
    (copy-calibrated), or None when there is none or the kernel sources have
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"kernel sources sha256 \(hog_kernels.hip \+ hog_internal.h\): ([0-9a-f]{64})", text)
    t = re.search(r"integral_emit<%d> traffic per launch: (\d+) bytes" % bin_chunk, text)
    if not h or not t or h.group(1) != kernel_sources_sha256():
        return None
    return int(t.group(1))


def path_bytes_per_pixel(wl, templates):
    """Algorithmic HBM bytes per processed pixel of one pass of the path: the
    image (C), the bin map written and read (2), the integral images written
    (4 N_b) and read at the cell corners (4 N_b / 64), the cell histograms
    (4 N_b / 64) and the scores (4 K / 64), per 8 x 8 cell of every level.
    Narrow planes scale the plane terms by their element size."""
    eb = wl.get("plane_bits", 32) // 8
    nb = wl["n_bins"]
    return wl["channels"] + 2 + eb * nb * (1 + 1 / 64) + 4 * nb / 64 + 4 * templates / 64


def batch_sizes(wl):
    import numpy as np
    rng = np.random.default_rng(wl["size_seed"])
    return [(int(rng.integers(320, 1921)), int(rng.integers(240, 1081))) for _ in range(wl["batch"])]


def workload_inputs(wl):
    """A workload's plan, its host images, the flat host input the step reads
    (the image, or the batch packed as the plan says) and its templates and
    biases, all seeded."""
    import numpy as np
    from paper_1703_06256_amd import hog, inputs
    kw = dict(channels=wl["channels"], n_bins=wl["n_bins"], max_levels=wl["max_levels"], scale=wl["scale"],
              norm=wl["norm"], n_templates=wl.get("templates", 1), plane_bits=wl.get("plane_bits", 32),
              votes=wl.get("votes", 0))
    if "batch" in wl:
        sizes = batch_sizes(wl)
        plan = hog.Plan([hog.make_desc(w, h, **kw) for w, h in sizes], batch=True)
        imgs = [inputs.synth_image(w, h, wl["channels"], wl["seed"] + j) for j, (w, h) in enumerate(sizes)]
        host = hog.pack_images(plan, imgs)
    else:
        plan = hog.Plan(hog.make_desc(wl["width"], wl["height"], **kw))
        imgs = [inputs.synth_image(wl["width"], wl["height"], wl["channels"], wl["seed"])]
        host = np.ascontiguousarray(imgs[0].reshape(-1))
    tmpl, bias = inputs.synth_templates(kw["n_templates"], plan.sizes.feature_dim, wl["tseed"])
    return plan, imgs, host, tmpl, bias


def oracle_units(wl):
    """The independent units of one step's oracle sample: (image index, level)
    pairs -- every level of the image, or of the first images of a batch."""
    if "batch" in wl:
        sizes = batch_sizes(wl)[:2]
    else:  # one image, or several distinct ones for a small workload
        sizes = [(wl["width"], wl["height"])] * wl.get("oracle_images", 1)
    import oracle
    units = []
    for j, (w, h) in enumerate(sizes):
        n = len(oracle.pyramid(w, h, wl["scale"], 64, 128, wl["max_levels"])) if wl["max_levels"] != 1 else 1
        units += [(j, w, h, l) for l in range(n)]
    return units


def oracle_unit(args):
    """The oracle over one level of one image: bins (FP64 angle), Eq. 5
    integral images, brute-force window scores; returns processed pixels.
    Runs in the bench process or in a worker process."""
    import oracle
    from paper_1703_06256_amd import inputs
    name, j, w, h, l = args
    wl = WORKLOADS[name]
    img = inputs.synth_image(w, h, wl["channels"], wl["seed"] + j)
    tmpl, bias = inputs.synth_templates(wl.get("templates", 1), oracle_dim(wl), wl["tseed"])
    p = oracle.ScanParams(norm=wl["norm"])
    nb = wl["n_bins"]
    if l == 0:
        lw, lh, lvl = w, h, img
    else:
        lw, lh, s = oracle.pyramid(w, h, wl["scale"], 64, 128, wl["max_levels"])[l]
        lvl = oracle.resize_nn(img, s, lw, lh)
    bins = oracle.bin_map(lvl, nb)
    oracle.integral(bins, nb)
    nwx, _ = oracle.window_grid(lw, lh, p)
    if nwx:
        oracle.score_windows(bins, nb, p, tmpl, bias)
    return lw * lh


def oracle_dim(wl):
    import oracle
    return oracle.ScanParams(norm=wl["norm"]).dim(wl["n_bins"])


def host_cpu():
    """(threads this process may run on, capped at the machine's CPU share, and the
    CPU model)."""
    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit():
        n = min(n, int(cap))
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


def cpu_baseline(name):
    """The oracle over one full step of the workload (batches: its first two
    images), timed single-threaded, then split by level across worker
    processes on the host cores. Run before the GPU is touched."""
    import concurrent.futures as cf
    import multiprocessing as mp
    wl = WORKLOADS[name]
    units = [(name,) + u for u in oracle_units(wl)]
    t0 = time.perf_counter()
    px = sum(oracle_unit(u) for u in units)
    dt1 = time.perf_counter() - t0
    n, model = host_cpu()
    workers = max(1, min(n, len(units)))
    # Largest levels first so that the pool ends together.
    order = sorted(units, key=lambda u: -(u[2] * u[3]) / wl["scale"] ** (2 * u[4]))
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(oracle_unit, [units[-1]] * workers))  # start the workers
        t0 = time.perf_counter()
        px_all = sum(ex.map(oracle_unit, order))
        dtn = time.perf_counter() - t0
    n_img = len({u[1] for u in units})
    what = (f"the first 2 images of the batch ({len(units)} levels, {px} processed pixels)" if "batch" in wl else
            f"one full step ({len(units)} levels, {px} processed pixels)" if n_img == 1 else
            f"{n_img} distinct images of the workload ({px} processed pixels)")
    return dict(value=round(px_all / dtn / 1e6, 3), unit="Mpixel/s", cores=workers, kind="oracle",
                sample=f"{what}: FP64 bins, Eq. 5 integrals, brute-force window scores; levels split "
                       f"across {workers} worker processes, {dtn:.2f} s",
                single_thread=dict(value=round(px / dt1 / 1e6, 3), cores=1, seconds=round(dt1, 2)),
                host=dict(cpu_model=model, threads_available=len(os.sched_getaffinity(0))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="pyramid_1920x1080", choices=sorted(WORKLOADS) + ["serve"])
    ap.add_argument("--rate", type=float, default=2000.0,
                    help="serve: offered load in requests per second (Poisson)")
    ap.add_argument("--requests", type=int, default=4000, help="serve: requests in the stream")
    ap.add_argument("--ring-bytes", type=float, default=float(1 << 30),
                    help="distinct buffer sets cycled through by the timed steps, at least this many "
                         "bytes in all (so that small workloads are timed from HBM, not the last-level cache)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lut", choices=("auto", "lds", "l2"), default="auto",
                    help="where the bin map reads the lookup table: as the autotuner picks, the LDS "
                         "half table, or the full table through L2")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(each image's path is independent, so images shard across GPUs without any "
              "exchange; no multi-GPU run is part of this benchmark).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # The oracle on the host cores, before anything touches the GPU (its
    # worker processes are started from a process that has not used HIP).
    cpu = None
    if not args.no_cpu_baseline and args.workload != "serve":
        cpu = cpu_baseline(args.workload)

    import torch
    from paper_1703_06256_amd import hog, inputs

    torch.cuda.set_device(0)
    if args.workload == "serve":
        from paper_1703_06256_amd import serving_bench
        r = serving_bench.measure(args.rate, args.requests)
        srv = r["server"]
        plain = r["per_image"]
        print(json.dumps({
            "metric": METRIC, "value": srv["mpixel_per_s"], "unit": "Mpixel/s", "n_gpus": 1,
            "steps": args.requests, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "serve", "requests": args.requests,
                       "offered_requests_per_s": args.rate,
                       "sizes": "320x240:800x600:1920x1080:3840x2160 = 4:3:2:1 (seed 5000)",
                       "n_bins": 8, "templates": serving_bench.K, "levels": 1, "norm": "l2",
                       "streams": r["streams"], "max_batch": r["max_batch"],
                       "copy_threads": r["copy_threads"]},
            "p50_ms": srv["p50_ms"], "p99_ms": srv["p99_ms"], "server": srv, "per_image": plain,
            "speedup_vs_per_image": round(srv["mpixel_per_s"] / plain["mpixel_per_s"], 3)}),
            flush=True)
        return
    wl = WORKLOADS[args.workload]
    batch = "batch" in wl
    K = wl.get("templates", 1)
    plan, imgs, host_img, tmpl, bias = workload_inputs(wl)
    img_t = torch.from_numpy(host_img).cuda()
    sz = plan.sizes
    lut = hog.hog_lut_build(wl["n_bins"])
    tmpl_t = torch.from_numpy(tmpl.reshape(-1)).cuda()
    bias_t = torch.from_numpy(bias).cuda()
    buf = hog.Buffers(plan)
    stream = torch.cuda.current_stream()

    # Tile shapes picked by timing candidates on these buffers.
    tiles = hog.autotune(plan, lut, img_t, tmpl_t, bias_t, buf, stream, reps=10)
    if args.lut != "auto":
        hog.set_plan_tiles(plan, tiles.bin_chunk, tiles.score_rows, tiles.level_groups,
                           lut_global=1 if args.lut == "l2" else 0)
        tiles = hog.plan_tiles(plan)

    # A ring of distinct buffer sets (input, bins, planes, scores, workspace)
    # of at least --ring-bytes in all: consecutive steps never find their
    # data in the last-level cache, whatever the workload's size.
    set_bytes = (img_t.numel() + sz.bins_bytes + sz.ii_elems * sz.ii_elem_bytes + 4 * sz.score_elems
                 + sz.workspace_bytes)
    n_sets = max(1, min(1024, -(-int(args.ring_bytes) // set_bytes)))
    sets = [(img_t, buf)]
    for _ in range(n_sets - 1):
        sets.append((img_t.clone(), hog.Buffers(plan)))
    ring = [0]
    if batch:
        graphs = [hog.Graph(plan, lut, im, tmpl_t, bias_t, b) for im, b in sets]
        graph = graphs[0]

        def step():
            graphs[ring[0] % n_sets].launch(stream)
            ring[0] += 1
    else:
        def step():
            im, b = sets[ring[0] % n_sets]
            hog.hog_run(plan, lut, im, tmpl_t, bias_t, b, stream)
            ring[0] += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Timed region: exactly K steps.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    value = sz.total_pixels / (ms_per_step * 1e3)

    # Per-step latency (each step alone between two events).
    lat = []
    n_lat = max(200, min(args.steps, 2000))
    for _ in range(n_lat):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b))
    lat = np.array(lat)

    # Per-kernel times: HIP event pairs recorded by the library around each
    # launch, on the launch stream. Taken on the three calls, which launch
    # each kernel once over all levels whatever the level groups, so every
    # kernel is timed alone at the plan's full size.
    hog.hog_timing_enable(True)
    hog.hog_timing_reset()
    n_k = max(min(args.steps, 200), min(50, 4 * n_sets))
    for i in range(n_k):
        im, b = sets[i % n_sets]
        hog.run_path(plan, lut, im, tmpl_t, bias_t, b, stream)  # eager: a graph records no events
    torch.cuda.synchronize()
    kern_us = {}
    for k in KERNELS:
        n, tot = hog.hog_timing_get(k)
        if n:
            kern_us[k] = round(tot / n * 1e3, 2)
    hog.hog_timing_enable(False)

    # Beside the device-resident rate: the same steps with the input first
    # copied from pinned host memory on the same stream (the PCIe-inclusive
    # rate; never `value`, the boundary takes device pointers).
    host_in = torch.empty(img_t.numel(), dtype=torch.uint8).pin_memory()
    host_in.copy_(img_t.cpu())
    n_h = min(args.steps, 50)
    for _ in range(3):
        img_t.copy_(host_in, non_blocking=True)
        step()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    # Both copy figures are the median of H2D_PASSES timed passes; a single
    # pass now and then runs about three times slower (on the small images,
    # where a pass lasts a few milliseconds), so every pass is reported too.
    h2d_passes = []
    for _ in range(H2D_PASSES):
        a.record(stream)
        for _ in range(n_h):
            img_t.copy_(host_in, non_blocking=True)
            step()
        b.record(stream)
        torch.cuda.synchronize()
        h2d_passes.append(a.elapsed_time(b) / n_h)
    h2d_ms = float(np.median(h2d_passes))
    with_h2d = dict(ms_per_step=round(h2d_ms, 5), mpixel_per_s=round(sz.total_pixels / (h2d_ms * 1e3), 1),
                    passes_ms=[round(t, 5) for t in h2d_passes], input_bytes=int(img_t.numel()))

    # The same with the copies overlapped: two streams, each with its own
    # input and buffer set, take alternate steps; on each, a step's copy
    # follows that stream's previous step, so one stream's copy runs while
    # the other computes. No step waits on another stream: the two streams
    # join the launch stream only at the ends of the timed region.
    ov_streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ov_sets = [sets[j] if j < n_sets else (img_t.clone(), hog.Buffers(plan)) for j in range(2)]
    ov_ins = [torch.empty_like(img_t) for _ in range(2)]
    if batch:
        ov_graphs = [hog.Graph(plan, lut, ov_ins[j], tmpl_t, bias_t, ov_sets[j][1]) for j in range(2)]

    def overlapped(n):
        for i in range(n):
            j = i & 1
            with torch.cuda.stream(ov_streams[j]):
                ov_ins[j].copy_(host_in, non_blocking=True)
                if batch:
                    ov_graphs[j].launch(ov_streams[j])
                else:
                    hog.hog_run(plan, lut, ov_ins[j], tmpl_t, bias_t, ov_sets[j][1], ov_streams[j])

    def joined(n):
        a.record(stream)
        for st in ov_streams:
            st.wait_event(a)
        overlapped(n)
        for st in ov_streams:
            e = torch.cuda.Event()
            e.record(st)
            stream.wait_event(e)
        b.record(stream)

    joined(4)
    torch.cuda.synchronize()
    ov_passes = []
    for _ in range(H2D_PASSES):
        joined(n_h)
        torch.cuda.synchronize()
        ov_passes.append(a.elapsed_time(b) / n_h)
    ov_ms = float(np.median(ov_passes))
    with_h2d["overlapped"] = dict(ms_per_step=round(ov_ms, 5),
                                  mpixel_per_s=round(sz.total_pixels / (ov_ms * 1e3), 1),
                                  passes_ms=[round(t, 5) for t in ov_passes])
    if batch:
        for g in ov_graphs:
            g.destroy()
    del ov_ins, ov_sets

    # The input's bin statistics (level 0 of the first image): every bin
    # populated and a visible no-bin share mean a non-degenerate workload.
    li0 = plan.levels[0]
    b0 = hog.level_bins(plan, buf.bins.cpu().numpy(), 0)
    b0 = b0[0] if isinstance(b0, tuple) else b0
    counts = np.bincount(b0.reshape(-1), minlength=256)
    bin_stats = dict(level0=f"{li0.width}x{li0.height}",
                     no_bin_fraction=round(float(counts[255]) / b0.size, 4),
                     histogram=[int(c) for c in counts[:wl["n_bins"]]])

    # Roofline of the dominant kernel: the integral-image writer moves, per
    # processed pixel, N_b plane elements of ii_elem_bytes (4 for uint32
    # planes) written and 1 byte of bins read.
    # With soft votes the writer is the weighted integral (two passes over
    # the planes); its algorithmic bytes are the planes written once and the
    # 2-byte soft bins read.
    soft = wl.get("votes", 0) == 1
    emit_kernel = "integral_soft" if soft else "integral_emit"
    emit_bytes = sz.total_pixels * (sz.ii_elem_bytes * wl["n_bins"] + (2 if soft else 1))
    extra = {}
    if batch:
        # The same images through 64 single-image plans, launched one image
        # after another (eager), and the batch plan launched eagerly.
        singles = []
        for j in range(len(imgs)):
            p1 = hog.Plan(plan.descs[j])
            b1 = hog.Buffers(p1)
            singles.append((p1, torch.from_numpy(imgs[j].reshape(-1)).cuda(), b1))

        def per_image():
            for p1, im1, b1 in singles:
                hog.hog_run(p1, lut, im1, tmpl_t, bias_t, b1, stream)

        def eager_batch():
            hog.hog_run(plan, lut, img_t, tmpl_t, bias_t, buf, stream)

        for name, fn in (("per_image", per_image), ("batch_eager", eager_batch)):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            reps = max(3, min(args.steps, 20))
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / reps
            extra[name] = dict(ms=round(t, 4), mpixel_per_s=round(sz.total_pixels / (t * 1e3), 1))
        extra["speedup_vs_per_image"] = round(extra["per_image"]["ms"] / ms_per_step, 3)
        del singles
    if "batched_form" in wl:
        # The same image size as one batch plan of many distinct images,
        # replayed as one captured graph: the batched form beside the
        # per-image launches above.
        nb_img = wl["batched_form"]
        kw = dict(channels=wl["channels"], n_bins=wl["n_bins"], max_levels=wl["max_levels"],
                  scale=wl["scale"], norm=wl["norm"], n_templates=K)
        bplan = hog.Plan([hog.make_desc(wl["width"], wl["height"], **kw)] * nb_img, batch=True)
        bimgs = [inputs.synth_image(wl["width"], wl["height"], wl["channels"], wl["seed"] + 10000 + j)
                 for j in range(nb_img)]
        bimg_t = torch.from_numpy(hog.pack_images(bplan, bimgs)).cuda()
        bbuf = hog.Buffers(bplan)
        btiles = hog.autotune(bplan, lut, bimg_t, tmpl_t, bias_t, bbuf, stream, reps=10)
        bgraph = hog.Graph(bplan, lut, bimg_t, tmpl_t, bias_t, bbuf)
        for _ in range(5):
            bgraph.launch(stream)
        torch.cuda.synchronize()
        blat = []
        for _ in range(200):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            bgraph.launch(stream)
            b.record(stream)
            b.synchronize()
            blat.append(a.elapsed_time(b))
        bms = float(np.mean(blat))
        bpx = bplan.sizes.total_pixels
        bbytes = path_bytes_per_pixel(wl, K) * bpx
        extra["batched_form"] = dict(
            images=nb_img, launch="one captured HIP graph of a batch plan", ms_per_batch=round(bms, 4),
            mpixel_per_s=round(bpx / (bms * 1e3), 1),
            speedup_vs_per_image=round(bpx / (bms * 1e3) / value, 3),
            p50_ms=round(float(np.percentile(blat, 50)), 4), p99_ms=round(float(np.percentile(blat, 99)), 4),
            path_frac=round(bbytes / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            tiles={"bin_chunk": btiles.bin_chunk, "score_rows": btiles.score_rows,
                   "level_groups": btiles.level_groups})
        bgraph.destroy()
        del bbuf, bimg_t
    if not batch:
        # The same steps with each buffer set's hog_run captured once into a
        # HIP graph and replayed over the same ring: what a caller that can
        # capture saves in launch overhead. `value` stays the plain per-call
        # rate above.
        pgraphs = [hog.Graph(plan, lut, im, tmpl_t, bias_t, b) for im, b in sets]
        for i in range(max(args.warmup, 3)):
            pgraphs[i % n_sets].launch(stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for i in range(args.steps):
            pgraphs[i % n_sets].launch(stream)
        b.record(stream)
        torch.cuda.synchronize()
        gms = a.elapsed_time(b) / args.steps
        extra["per_image_graph"] = dict(
            launch="hog_run captured into one HIP graph per buffer set", ms_per_step=round(gms, 5),
            mpixel_per_s=round(sz.total_pixels / (gms * 1e3), 1), buffer_sets=n_sets,
            speedup_vs_calls=round(ms_per_step / gms, 3))
        for g in pgraphs:
            g.destroy()
        del pgraphs

    # This GPU's plain 1 GiB copy (read + write) and fill (write only) rates,
    # timed the same way on the same stream: what a bandwidth-bound kernel
    # reaches in practice, beside the 8 TB/s peak.
    src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)

    def rate(fn, nbytes, reps=5):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9

    copy_gbs = rate(lambda: dst.copy_(src), 2 * 4 * src.numel())
    fill_gbs = rate(lambda: dst.fill_(7), 4 * dst.numel())
    del src, dst

    emit_us = kern_us.get(emit_kernel, float("nan"))
    achieved = emit_bytes / (emit_us * 1e-6) / 1e9
    traffic = None if soft else measured_traffic(args.workload, tiles.bin_chunk)
    roofline = dict(bound="hbm", kernel=emit_kernel, achieved=round(achieved, 1),
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=traffic, algorithmic_bytes_per_launch=emit_bytes,
                    measured=None if traffic is None else round(traffic / (emit_us * 1e-6) / 1e9, 1),
                    copy_GBps=round(copy_gbs, 1), fill_GBps=round(fill_gbs, 1),
                    frac_of_fill=round(achieved / fill_gbs, 4), frac_of_copy=round(achieved / copy_gbs, 4))
    if traffic is not None:
        roofline["measured_frac"] = round(roofline["measured"] / HBM_PEAK_GBS, 4)
        roofline["measured_frac_of_copy"] = round(roofline["measured"] / copy_gbs, 4)
    # The whole path: its algorithmic bytes per step over the step time.
    path_bytes = path_bytes_per_pixel(wl, K) * sz.total_pixels
    roofline["path_bytes_per_step"] = int(path_bytes)
    roofline["path_GBps"] = round(path_bytes / (ms_per_step * 1e-3) / 1e9, 1)
    roofline["path_frac"] = round(path_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    if args.copy_calibration:
        # A plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between those counters and bytes moved.
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {4: "u32", 2: "u16", 1: "u8"}[sz.ii_elem_bytes],
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "image": (f"{wl['batch']} images {wl['channels']}ch uint8, sizes uniform 320..1920 x "
                      f"240..1080 (seed {wl['size_seed']})") if batch else
                     f"{wl['width']}x{wl['height']}x{wl['channels']} uint8",
            "n_bins": wl["n_bins"],
            "levels": sz.n_levels,
            "pyramid_scale": wl["scale"],
            "processed_pixels": sz.total_pixels,
            "windows": sz.total_windows,
            "feature_dim": sz.feature_dim,
            "norm": "l2" if wl["norm"] else "raw",
            "templates": K,
            "plane_bits": 8 * sz.ii_elem_bytes,
            "votes": "soft (1/32)" if soft else "hard",
            "launch": "captured HIP graph of the batch plan" if batch else "hog_run per step",
            "buffer_sets": n_sets,
            "tiles": {"bin_chunk": tiles.bin_chunk, "score_rows": tiles.score_rows,
                      "level_groups": tiles.level_groups,
                      "lut": "full table through L2" if tiles.lut_global else "half table in LDS",
                      "how": "autotuned" if args.lut == "auto" else f"autotuned, table forced to {args.lut}"},
        },
        "base_mpixel_per_s": round(sum(d.width * d.height for d in plan.descs) / (ms_per_step * 1e3), 2) if batch
        else round(wl["width"] * wl["height"] / (ms_per_step * 1e3), 2),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "wall_ms_timed": round(wall_ms, 2),
        "kernel_us": kern_us,
        "with_h2d": with_h2d,
        "bins": bin_stats,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
