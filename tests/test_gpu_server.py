"""Serving (hog_server_*, hog_submit, hog_poll, hog_wait_any): requests of mixed sizes,
submitted while others run, each give the scores of their image run alone
(bit for bit) and of the oracle (within tolerance); a memory budget that
fits one request at a time still completes every request; bad calls fail
cleanly."""
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog
from paper_1703_06256_amd import inputs

from hog_cases import check_scores, oracle_params, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _torch_first():
    """The reference runs below use PyTorch for device buffers: initialise
    its runtime before the server starts its streams and worker thread."""
    import torch
    torch.cuda.init()
    torch.zeros(1, device="cuda")

K = 4
SIZES = [(320, 240), (200, 150), (641, 480), (123, 300), (800, 600), (64, 128), (70, 60)]


def _templates():
    dim = oracle_params(hog.make_desc(64, 128, n_bins=8, norm=hog.HOG_NORM_L2)).dim(8)
    return inputs.synth_templates(K, dim, 5050)


def _alone(img, tmpl, bias):
    h, w = img.shape[:2]
    desc = hog.make_desc(w, h, channels=3, n_bins=8, n_templates=K, norm=hog.HOG_NORM_L2)
    plan, out = run_gpu(desc, img, tmpl, bias, cell_hist=False, block_feat=False)
    li = plan.levels[0]
    return hog.level_scores(plan, out["scores"], 0).reshape(-1), li.windows_x, li.windows_y


def _wait(srv, tickets, caps, timeout=60.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t, c in zip(tickets, caps):
            if t not in res:
                r = srv.poll(t, c)
                if r is not None:
                    res[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.001)
    return res


def _cap(w, h):
    return max(1, ((w // 8) - 7) * ((h // 8) - 15) * K)


def test_mixed_requests_equal_alone_and_oracle():
    tmpl, _ = _templates()
    bias = np.array([0.5, -1.0, 2.0, 0.0], np.float32)
    srv = hog.Server(tmpl, bias, channels=3, n_bins=8, max_width=800, max_height=600,
                     memory_budget=768 << 20, max_slots=8, max_batch=4, streams=3)
    rng = np.random.default_rng(5000)
    reqs = []
    # Two submitting threads, requests arriving while others run.
    def submit(idx):
        for j in idx:
            w, h = SIZES[j % len(SIZES)]
            img = inputs.synth_image(w, h, 3, 5000 + j)
            t = srv.submit(img)
            reqs.append((t, img, w, h))
            time.sleep(float(rng.uniform(0, 0.003)))
    th = [threading.Thread(target=submit, args=(range(k, 24, 2),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    res = _wait(srv, [r[0] for r in reqs], [_cap(r[2], r[3]) for r in reqs])
    for n, (t, img, w, h) in enumerate(reqs):
        scores, nwx, nwy, lat = res[t]
        want, wx, wy = _alone(img, tmpl, bias)
        assert (nwx, nwy) == (max(wx, 0), max(wy, 0))
        assert np.array_equal(scores.view(np.uint32), want.view(np.uint32)), f"request {n} {w}x{h}"
        assert lat > 0
        if n < 4 and nwx:
            bins = oracle.bin_map(img, 8)
            ref, absterm, _, _, _ = oracle.score_windows(bins, 8, oracle_params(
                hog.make_desc(w, h, n_bins=8, norm=hog.HOG_NORM_L2)), tmpl, bias)
            check_scores(scores.reshape(ref.shape), ref, absterm)
    srv.close()


def test_budget_for_one_request_at_a_time_still_finishes_all():
    tmpl, bias = _templates()
    # The 800x600 request alone: a budget just above it admits one at a time.
    desc = hog.make_desc(800, 600, channels=3, n_bins=8, n_templates=K, norm=hog.HOG_NORM_L2)
    z = hog.Plan(desc).sizes
    need = z.bins_bytes + z.ii_elems * 4 + z.score_elems * 4 + z.workspace_bytes + 800 * 600 * 3
    srv = hog.Server(tmpl, bias, max_width=800, max_height=600, memory_budget=need + (1 << 16),
                     max_slots=8, max_batch=4, streams=2)
    imgs = [inputs.synth_image(800, 600, 3, 5300 + j) for j in range(5)]
    tickets = [srv.submit(im) for im in imgs]
    res = _wait(srv, tickets, [_cap(800, 600)] * 5)
    for t, im in zip(tickets, imgs):
        want, _, _ = _alone(im, tmpl, bias)
        assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32))
    srv.close()


def test_server_errors():
    tmpl, bias = _templates()
    srv = hog.Server(tmpl, bias, max_width=320, max_height=240, memory_budget=64 << 20)
    with pytest.raises(hog.HogError) as e:
        srv.poll(12345, 10)
    assert e.value.status == hog.HOG_E_INVALID
    with pytest.raises(hog.HogError) as e:
        srv.submit(inputs.synth_image(400, 240, 3, 1))
    assert e.value.status == hog.HOG_E_INVALID
    img = inputs.synth_image(320, 240, 3, 2)
    t = srv.submit(img)
    while True:
        try:
            r = srv.poll(t, 1)  # too small once ready
        except hog.HogError as err:
            assert err.status == hog.HOG_E_INVALID
            break
        assert r is None
        time.sleep(0.001)
    r = srv.poll(t, _cap(320, 240))  # the request was kept
    want, _, _ = _alone(img, tmpl, bias)
    assert np.array_equal(r[0].view(np.uint32), want.view(np.uint32))
    srv.close()
    with pytest.raises(hog.HogError):
        hog.Server(tmpl, bias, max_batch=0)


def test_wait_any_reports_each_ticket_once():
    tmpl, bias = _templates()
    srv = hog.Server(tmpl, bias, channels=3, n_bins=8, max_width=800, max_height=600,
                     memory_budget=512 << 20, max_slots=8, max_batch=4, streams=2)
    srv.warm(320, 240)
    sizes = [SIZES[j % 3] for j in range(12)]
    imgs = [inputs.synth_image(w, h, 3, 5400 + j) for j, (w, h) in enumerate(sizes)]
    tickets = [srv.submit(im) for im in imgs]
    seen = []
    t0 = time.time()
    while len(seen) < len(tickets):
        seen += srv.wait_any(2000)
        assert time.time() - t0 < 60, "requests did not finish"
    assert sorted(seen) == sorted(tickets)
    assert srv.wait_any(0) == []
    for t, im, (w, h) in zip(tickets, imgs, sizes):
        r = srv.poll(t, _cap(w, h))
        assert r is not None
        want, _, _ = _alone(im, tmpl, bias)
        assert np.array_equal(r[0].view(np.uint32), want.view(np.uint32))
    with pytest.raises(hog.HogError) as e:
        srv.warm(801, 600)
    assert e.value.status == hog.HOG_E_INVALID
    srv.close()


def test_host_budget_rejects_with_busy_and_accepted_requests_finish():
    tmpl, bias = _templates()
    one = 320 * 240 * 3
    with pytest.raises(hog.HogError) as e:
        hog.Server(tmpl, bias, max_width=320, max_height=240, memory_budget=64 << 20,
                   host_budget=one - 1)
    assert e.value.status == hog.HOG_E_INVALID
    srv = hog.Server(tmpl, bias, max_width=320, max_height=240, memory_budget=64 << 20,
                     host_budget=2 * 256 * ((one + 255) // 256), max_slots=4, max_batch=2)
    imgs = [inputs.synth_image(320, 240, 3, 5500 + j) for j in range(16)]
    accepted = []
    for im in imgs:
        try:
            accepted.append((srv.submit(im), im))
        except hog.HogError as err:
            assert err.status == hog.HOG_E_BUSY
    assert accepted
    res = _wait(srv, [t for t, _ in accepted], [_cap(320, 240)] * len(accepted))
    for t, im in accepted:
        want, _, _ = _alone(im, tmpl, bias)
        assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32))
    srv.close()


def test_unpolled_results_hold_output_space_until_polled():
    """Finished results wait in a pinned output arena of 2 * max_slots
    results: a client that lets 4 pile up sees admission pause, never more
    than 4 unpolled, and every request finishes once it polls."""
    tmpl, bias = _templates()
    srv = hog.Server(tmpl, bias, max_width=320, max_height=240, memory_budget=256 << 20,
                     max_slots=2, max_batch=2, streams=2)
    imgs = [inputs.synth_image(320, 240, 3, 5600 + j) for j in range(10)]
    tickets = [srv.submit(im) for im in imgs]
    unpolled, res = [], {}
    t0 = time.time()
    while len(res) < len(tickets):
        unpolled += srv.wait_any(2000)
        assert len(unpolled) <= 4
        if len(unpolled) == 4 or len(unpolled) + len(res) == len(tickets):
            time.sleep(0.02)  # no room for another result meanwhile
            unpolled += srv.wait_any(0)
            assert len(unpolled) <= 4
            for t in unpolled:
                res[t] = srv.poll(t, _cap(320, 240))
            unpolled = []
        assert time.time() - t0 < 60, "requests did not finish"
    for t, im in zip(tickets, imgs):
        want, _, _ = _alone(im, tmpl, bias)
        assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32))
    srv.close()


def test_large_images_copied_in_pieces_equal_alone():
    """Images above 2 MiB are copied into the server by the caller and
    helper threads together (copy_threads); two submitting threads share
    the helpers."""
    tmpl, bias = _templates()
    with pytest.raises(hog.HogError) as e:
        hog.Server(tmpl, bias, copy_threads=33)
    assert e.value.status == hog.HOG_E_INVALID
    srv = hog.Server(tmpl, bias, max_width=1920, max_height=1080, memory_budget=1 << 30,
                     max_slots=8, max_batch=4, streams=2, copy_threads=3)
    sizes = [(1920, 1080), (1000, 700), (1283, 721), (1920, 1080)]
    imgs = [inputs.synth_image(w, h, 3, 5700 + j) for j, (w, h) in enumerate(sizes * 2)]
    got = [None] * len(imgs)

    def submit(idx):
        for j in idx:
            got[j] = srv.submit(imgs[j])
    th = [threading.Thread(target=submit, args=(range(k, len(imgs), 2),)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    res = _wait(srv, got, [_cap(im.shape[1], im.shape[0]) for im in imgs])
    for t, im in zip(got, imgs):
        want, _, _ = _alone(im, tmpl, bias)
        assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32))
    srv.close()


@pytest.mark.parametrize("votes,plane_bits", [(hog.HOG_VOTES_HARD, 8), (hog.HOG_VOTES_SOFT, 32)])
def test_server_votes_and_plane_bits(votes, plane_bits):
    """The server's plans take the configured votes and plane element; the
    scores equal a single-image plan of the same description (and, for
    8-bit planes, the uint32 plan: the scores never read the planes)."""
    import torch
    tmpl, bias = _templates()
    srv = hog.Server(tmpl, bias, max_width=800, max_height=600, memory_budget=512 << 20,
                     votes=votes, plane_bits=plane_bits)
    sizes = [(320, 240), (641, 480), (800, 600)]
    imgs = [inputs.synth_image(w, h, 3, 5800 + j) for j, (w, h) in enumerate(sizes)]
    tickets = [srv.submit(im) for im in imgs]
    res = _wait(srv, tickets, [_cap(w, h) for w, h in sizes])
    srv.close()
    for t, im, (w, h) in zip(tickets, imgs, sizes):
        for pb in {plane_bits, 32}:
            desc = hog.make_desc(w, h, channels=3, n_bins=8, n_templates=K, norm=hog.HOG_NORM_L2,
                                 votes=votes, plane_bits=pb)
            plan, out = run_gpu(desc, im, tmpl, bias, cell_hist=False, block_feat=False)
            want = hog.level_scores(plan, out["scores"], 0).reshape(-1)
            assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32)), (w, h, pb)
    torch.cuda.synchronize()


def test_many_distinct_sizes_past_the_plan_cache_bound():
    """More distinct image sizes than the server caches plans for (4 max_batch
    + 16 = 24 with max_batch 2): plans are dropped and rebuilt as sizes
    return, and every request still equals its image run alone."""
    tmpl, bias = _templates()
    srv = hog.Server(tmpl, bias, channels=3, n_bins=8, max_width=224, max_height=248,
                     memory_budget=256 << 20, host_budget=64 << 20, max_slots=4, max_batch=2, streams=2)
    sizes = [(64 + 4 * i, 128 + 3 * i) for i in range(40)]
    order = sizes + sizes[::-3]  # some sizes come back after their plans were dropped
    reqs = []
    for j, (w, h) in enumerate(order):
        img = inputs.synth_image(w, h, 3, 7700 + j)
        reqs.append((srv.submit(img), img, w, h))
    res = _wait(srv, [r[0] for r in reqs], [_cap(r[2], r[3]) for r in reqs])
    for t, img, w, h in reqs:
        want, _, _ = _alone(img, tmpl, bias)
        assert np.array_equal(res[t][0].view(np.uint32), want.view(np.uint32)), f"{w}x{h}"
    srv.close()
