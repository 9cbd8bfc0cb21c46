"""Host-side parts of bench.py that run without a GPU: the one-GPU guard,
the workload recipes, and the traffic lookup that ties roofline.traffic to
the committed counter summary of the current kernel sources."""
import os
import re
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batch64_sizes_follow_the_recipe():
    wl = bench.WORKLOADS["batch64"]
    sizes = bench.batch_sizes(wl)
    assert len(sizes) == 64
    assert all(320 <= w <= 1920 and 240 <= h <= 1080 for w, h in sizes)
    assert sizes == bench.batch_sizes(wl)  # seeded: the same every time
    assert len(set(sizes)) > 60  # uneven sizes, not one repeated shape


def test_workloads_name_what_the_bench_reads():
    for name, wl in bench.WORKLOADS.items():
        for key in ("channels", "n_bins", "max_levels", "scale", "norm", "seed", "tseed"):
            assert key in wl, (name, key)
        assert ("batch" in wl) == ("width" not in wl), name
        assert wl.get("plane_bits", 32) in (32, 16, 8)
        assert wl.get("votes", 0) in (0, 1)


def test_traffic_lookup_matches_the_committed_summary():
    path = os.path.join(ROOT, "profiles", "hbm_traffic_pyramid_1920x1080.txt")
    text = open(path).read()
    recorded = re.search(r"kernel sources sha256 \(hog_kernels.hip \+ hog_internal.h\): ([0-9a-f]{64})", text)
    assert recorded, "the summary records the kernel sources it was taken on"
    if recorded.group(1) != bench.kernel_sources_sha256():
        # Kernels changed since the counters were taken: the bench must then
        # report no traffic rather than a stale figure.
        assert all(bench.measured_traffic("pyramid_1920x1080", c) is None for c in range(1, 7))
        return
    algorithmic = 21970720 * (4 * 18 + 1)
    for c in range(2, 7):
        t = bench.measured_traffic("pyramid_1920x1080", c)
        assert t is not None and algorithmic <= t < 1.2 * algorithmic, (c, t)
    assert bench.measured_traffic("pyramid_1920x1080", 1) is None  # not a candidate the autotuner runs
    assert bench.measured_traffic("no_such_workload", 6) is None


def test_path_bytes_per_pixel_follow_the_cost_model():
    """C + 2 + 4 N_b (1 + 1/64) + 4 N_b / 64 + 4 K / 64 bytes per processed pixel."""
    assert abs(bench.path_bytes_per_pixel(bench.WORKLOADS["pyramid_1920x1080"], 1) - 79.3125) < 1e-9
    assert abs(bench.path_bytes_per_pixel(bench.WORKLOADS["gray_320x240"], 1) - 36.0625) < 1e-9
    assert abs(bench.path_bytes_per_pixel(bench.WORKLOADS["rgb_800x600"], 1) - 38.0625) < 1e-9
    u16 = bench.path_bytes_per_pixel(bench.WORKLOADS["pyramid_1920x1080_u16"], 1)
    assert abs(u16 - (5 + 2 * 18 * (1 + 1 / 64) + 72 / 64 + 4 / 64)) < 1e-9


def test_oracle_units_cover_every_level():
    units = bench.oracle_units(bench.WORKLOADS["pyramid_1920x1080"])
    assert len(units) == 44 and [u[3] for u in units] == list(range(44))
    small = bench.oracle_units(bench.WORKLOADS["gray_320x240"])
    assert small == [(j, 320, 240, 0) for j in range(192)]  # distinct seeded images
    assert len({u[0] for u in bench.oracle_units(bench.WORKLOADS["batch64"])}) == 2


def test_cpu_baseline_reports_both_modes_and_the_host():
    r = bench.cpu_baseline("gray_320x240")
    assert r["kind"] == "oracle" and r["unit"] == "Mpixel/s" and r["value"] > 0
    assert r["cores"] >= 1 and r["single_thread"]["cores"] == 1 and r["single_thread"]["value"] > 0
    assert r["host"]["cpu_model"] and r["host"]["threads_available"] >= 1
