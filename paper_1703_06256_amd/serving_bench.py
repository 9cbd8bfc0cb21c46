"""Serving measurement: a Poisson stream of requests through hog_server
(continuous batching) and, for comparison, through the plain per-image path
(one request at a time: copy in, hog_run on its own plan, copy out).

Requests: RGB uint8 images with sizes drawn from {320x240, 800x600,
1920x1080, 3840x2160} in proportions 4:3:2:1 (seeded), N_b = 8, L2 blocks,
K = 4 templates, single level. Throughput counts the pixels of completed
requests over the time from the first arrival to the last completion;
latency runs from a request's arrival to its completion. Each path serves
the stream twice and reports the second pass.

The server's client has two threads, one submitting at the arrival times
and one taking completions from hog_wait_any; the server runs `streams`
batches at once, up to max_batch requests of one size each, and splits the
copy of large images over copy_threads helpers.
"""
from __future__ import annotations

import threading
import time

import numpy as np

SIZES = [(320, 240), (800, 600), (1920, 1080), (3840, 2160)]
WEIGHTS = [4, 3, 2, 1]
K = 4


def request_stream(n: int, rate: float, seed: int):
    """(arrival time s, (w, h), image seed) for n requests at `rate` per second."""
    rng = np.random.default_rng(seed)
    p = np.array(WEIGHTS, float) / sum(WEIGHTS)
    kinds = rng.choice(len(SIZES), size=n, p=p)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[i]), SIZES[kinds[i]], seed + 1 + i) for i in range(n)]


def _images(stream):
    from paper_1703_06256_amd import inputs
    cache = {}
    out = []
    for _, (w, h), s in stream:
        # a few distinct images per size keep the host side cheap
        key = (w, h, s % 4)
        if key not in cache:
            cache[key] = inputs.synth_image(w, h, 3, 5000 + len(cache))
        out.append(cache[key])
    return out


def _pct(x, q):
    return round(float(np.percentile(np.asarray(x), q)) * 1e3, 3)


def _summary(stream, done, t0):
    lat = [done[i][0] - (t0 + stream[i][0]) for i in range(len(stream))]
    px = sum(w * h for _, (w, h), _ in stream)
    span = max(d[0] for d in done.values()) - t0
    return dict(mpixel_per_s=round(px / span / 1e6, 1), requests_per_s=round(len(stream) / span, 1),
                p50_ms=_pct(lat, 50), p99_ms=_pct(lat, 99))


def run_server(stream, imgs, tmpl, bias, **cfg):
    from paper_1703_06256_amd import hog
    srv = hog.Server(tmpl, bias, channels=3, n_bins=8, max_width=3840, max_height=2160, **cfg)
    caps = {wh: max(1, ((wh[0] // 8) - 7) * ((wh[1] // 8) - 15) * K) for wh in SIZES}
    outs = {wh: np.empty(caps[wh], np.float32) for wh in SIZES}
    # build the batch plans of every size, then one request per size end to end
    for wh in SIZES:
        srv.warm(*wh)
        t = srv.submit(np.zeros((wh[1], wh[0], 3), np.uint8))
        while srv.poll(t, caps[wh], outs[wh]) is None:
            time.sleep(0.0005)
    while srv.wait_any(0):  # the warm-up tickets
        pass
    out = _serve_once(srv, stream, imgs, caps)  # untimed: first use of the arenas and threads
    out = _serve_once(srv, stream, imgs, caps)
    srv.close()
    return out


def _serve_once(srv, stream, imgs, caps):
    from paper_1703_06256_amd import hog
    # One thread submits at the arrival times, another takes completions
    # (the library releases the interpreter lock in both calls).
    n = len(stream)
    cap = max(caps.values())
    got = {}  # ticket -> (time the client had the scores, server latency)
    stop = threading.Event()

    def completions():
        out = np.empty(cap, np.float32)
        while len(got) < n and not stop.is_set():
            for t in srv.wait_any(2000):
                r = srv.poll(t, cap, out)
                got[t] = (time.perf_counter(), r[3])

    tickets = [0] * n
    submitted = [0.0] * n  # when hog_submit returned
    th = threading.Thread(target=completions)
    t0 = time.perf_counter()
    th.start()
    busy = 0
    try:
        for i in range(n):
            d = t0 + stream[i][0] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            while True:  # back off while the server's queue or pinned memory is full
                try:
                    tickets[i] = srv.submit(imgs[i])
                    break
                except hog.HogError as e:
                    if e.status != hog.HOG_E_BUSY:
                        raise
                    busy += 1
                    time.sleep(0.0002)
            submitted[i] = time.perf_counter()
    except BaseException:
        stop.set()
        raise
    finally:
        th.join()
    done = {i: got[tickets[i]] for i in range(n)}
    out = _summary(stream, done, t0)
    # Where a request's latency goes: the client's submission running late
    # (arrival to hog_submit's return), the server (hog_submit to completion,
    # its own clock) and the client noticing (completion to hog_poll).
    lag = [submitted[i] - (t0 + stream[i][0]) for i in range(n)]
    srv_lat = [done[i][1] for i in range(n)]
    report = [done[i][0] - submitted[i] - done[i][1] for i in range(n)]
    out.update(submit_lag_p50_ms=_pct(lag, 50), submit_lag_p99_ms=_pct(lag, 99),
               server_latency_p50_ms=_pct(srv_lat, 50), server_latency_p99_ms=_pct(srv_lat, 99),
               report_lag_p99_ms=_pct(report, 99), busy_retries=busy)
    return out


def run_per_image(stream, imgs, tmpl, bias):
    import torch
    from paper_1703_06256_amd import hog
    lut = hog.hog_lut_build(8)
    tt = torch.from_numpy(np.ascontiguousarray(tmpl).reshape(-1)).cuda()
    bt = torch.from_numpy(bias).cuda()
    per = {}
    for wh in SIZES:
        plan = hog.Plan(hog.make_desc(wh[0], wh[1], channels=3, n_bins=8, n_templates=K,
                                      norm=hog.HOG_NORM_L2))
        per[wh] = (plan, hog.Buffers(plan, cell_hist=False, block_feat=False),
                   torch.empty(wh[0] * wh[1] * 3, dtype=torch.uint8).pin_memory(),
                   torch.empty(wh[0] * wh[1] * 3, dtype=torch.uint8, device="cuda"),
                   torch.empty(max(plan.sizes.score_elems, 1), dtype=torch.float32).pin_memory())
    stream_ = torch.cuda.current_stream()
    for wh, (plan, buf, hin, din, hout) in per.items():  # warm up
        hog.hog_run(plan, lut, din, tt, bt, buf)
    torch.cuda.synchronize()
    for _ in range(2):  # the first pass untimed, as for the server
        done = {}
        t0 = time.perf_counter()
        for i, (ta, wh, _) in enumerate(stream):
            while time.perf_counter() - t0 < ta:
                pass
            plan, buf, hin, din, hout = per[wh]
            hin.numpy()[:] = imgs[i].reshape(-1)
            din.copy_(hin, non_blocking=True)
            hog.hog_run(plan, lut, din, tt, bt, buf, stream_)
            n = plan.sizes.score_elems
            if n:
                hout[:n].copy_(buf.scores[:n], non_blocking=True)
            stream_.synchronize()
            done[i] = (time.perf_counter(), 0.0)
    return _summary(stream, done, t0)


def measure(rate: float, n: int = 400, seed: int = 5000, memory_budget: int = 8 << 30, streams: int = 3,
            max_batch: int = 16, host_budget: int = 2 << 30, copy_threads: int = 8):
    import torch
    torch.cuda.init()
    torch.zeros(1, device="cuda")
    from paper_1703_06256_amd import hog, inputs
    stream = request_stream(n, rate, seed)
    imgs = _images(stream)
    dim = 105 * 4 * 8
    tmpl, bias = inputs.synth_templates(K, dim, 9004)
    srv = run_server(stream, imgs, tmpl, bias, memory_budget=memory_budget, host_budget=host_budget,
                     max_slots=32, max_batch=max_batch, streams=streams, copy_threads=copy_threads)
    plain = run_per_image(stream, imgs, tmpl, bias)
    return dict(offered_requests_per_s=rate, requests=n, streams=streams, max_batch=max_batch,
                copy_threads=copy_threads,
                server=srv, per_image=plain)
