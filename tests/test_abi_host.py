"""Host-side checks of libhog: it loads, exports every symbol the header
declares, builds the lookup table on the host exactly as the oracle bins,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hog.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hog_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    declared = _declared()
    assert set(declared) == set(hog.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", hog.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    lib = hog.load_library()
    for s in declared:
        assert getattr(lib, s) is not None


@pytest.mark.parametrize("nb", list(range(1, 65)))
def test_host_lut_equals_oracle_bins(nb):
    assert np.array_equal(hog.hog_lut_fill_host(nb), oracle.bin_table(nb))


def test_lut_fill_rejects_bad_bins():
    for nb in (0, -1, 65):
        with pytest.raises(hog.HogError) as e:
            hog.hog_lut_fill_host(nb)
        assert e.value.status == hog.HOG_E_INVALID


BAD_DESCS = [
    dict(width=0), dict(height=-3), dict(width=40000), dict(channels=2), dict(n_bins=0),
    dict(n_bins=65), dict(max_levels=-1), dict(max_levels=0, scale=1.0),
    dict(max_levels=3, scale=0.9), dict(n_templates=0), dict(cell=0), dict(cell=33),
    dict(win_cells_x=0), dict(win_cells_y=65), dict(norm=2),
    dict(norm=hog.HOG_NORM_L2, block=3), dict(norm=hog.HOG_NORM_L2, win_cells_x=1),
    dict(norm=hog.HOG_NORM_L2, eps=float("nan")),
    dict(plane_bits=12), dict(plane_bits=64), dict(plane_bits=-8),
    dict(plane_bits=8, cell=16), dict(plane_bits=8, cell=32),
    dict(votes=2), dict(votes=-1), dict(votes=1, plane_bits=16), dict(votes=1, plane_bits=8),
    dict(votes=1, width=32767, height=32767),
]


@pytest.mark.parametrize("bad", BAD_DESCS)
def test_plan_create_rejects_bad_descriptions(bad):
    args = dict(width=320, height=240, channels=1, n_bins=8)
    args.update(bad)
    desc = hog.make_desc(**args)
    lib = hog.load_library()
    h = ctypes.c_void_p()
    st = lib.hog_plan_create(ctypes.byref(desc), ctypes.byref(h))
    assert st == hog.HOG_E_INVALID
    assert not h.value
    assert lib.hog_last_error().decode()


def test_calls_reject_null_arguments():
    lib = hog.load_library()
    assert lib.hog_bin_map(None, None, None, 0, None, None) == hog.HOG_E_INVALID
    assert lib.hog_integral(None, None, None, None, None) == hog.HOG_E_INVALID
    assert lib.hog_scan_windows(None, None, None, None, None, None, None, None,
                                None) == hog.HOG_E_INVALID
    assert lib.hog_plan_create(None, None) == hog.HOG_E_INVALID
    assert lib.hog_lut_build(1, None) == hog.HOG_E_INVALID
    assert lib.hog_plan_get_sizes(None, None) == hog.HOG_E_INVALID
    assert "NULL" in lib.hog_last_error().decode()
    lib.hog_plan_destroy(None)
    lib.hog_lut_free(None)


@pytest.mark.parametrize("orientation", [hog.HOG_ORIENT_SIGNED, hog.HOG_ORIENT_UNSIGNED])
@pytest.mark.parametrize("nb", list(range(1, 65)))
def test_lut_mirror_rule_behind_the_half_table(nb, orientation):
    """The kernels keep only the dy >= 0 half of the table plus one flag:
    bin(dx, -dy) = nb - 1 - bin(dx, dy) + f with f in {0, 1}, f = 1 exactly on
    sector edges (where the mirrored angle 2 pi - t, or pi - t for unsigned
    orientation, is a multiple of the sector width)."""
    t = hog.hog_lut_fill_host(nb, orientation).astype(np.int64)
    up = t[255 + 1:, :]          # dy = 1..255
    dn = t[255 - 1::-1, :]       # dy = -1..-255
    f = dn - (nb - 1 - up)
    assert set(np.unique(f)) <= {0, 1}
    dxs = np.arange(-255, 256)[None, :]
    dys = np.arange(1, 256)[:, None]
    # an edge of the mirrored direction can only be an axis or a diagonal
    edge = (dxs == 0) | (np.abs(dxs) == dys)
    assert not f[~edge].any()


@pytest.mark.parametrize("bad", [dict(n_bins=9), dict(channels=1), dict(n_templates=2),
                                 dict(norm=hog.HOG_NORM_L2, cell=4), dict(plane_bits=16), dict(votes=1)])
def test_batch_plan_rejects_mismatched_images(bad):
    base = dict(width=320, height=240, channels=3, n_bins=8)
    other = dict(base, width=200, height=150)
    other.update(bad)
    descs = (hog.PlanDesc * 2)(hog.make_desc(**base), hog.make_desc(**other))
    lib = hog.load_library()
    h = ctypes.c_void_p()
    assert lib.hog_plan_create_batch(descs, 2, ctypes.byref(h)) == hog.HOG_E_INVALID
    assert not h.value
    assert "match image 0" in lib.hog_last_error().decode()


def test_batch_plan_rejects_bad_counts_and_bad_members():
    lib = hog.load_library()
    h = ctypes.c_void_p()
    one = (hog.PlanDesc * 1)(hog.make_desc(320, 240))
    assert lib.hog_plan_create_batch(one, 0, ctypes.byref(h)) == hog.HOG_E_INVALID
    assert lib.hog_plan_create_batch(None, 1, ctypes.byref(h)) == hog.HOG_E_INVALID
    bad = (hog.PlanDesc * 2)(hog.make_desc(320, 240), hog.make_desc(0, 240))
    assert lib.hog_plan_create_batch(bad, 2, ctypes.byref(h)) == hog.HOG_E_INVALID
    assert lib.hog_plan_images(None) == 0
    assert lib.hog_plan_get_image(None, 0, None) == hog.HOG_E_INVALID


@pytest.mark.parametrize("nb", list(range(1, 65)))
def test_unsigned_host_table_equals_oracle(nb):
    assert np.array_equal(hog.hog_lut_fill_host(nb, hog.HOG_ORIENT_UNSIGNED),
                          oracle.bin_table(nb, unsigned=True))


def test_lut_rejects_unknown_orientation():
    lib = hog.load_library()
    out = np.empty((511, 511), np.uint8)
    assert lib.hog_lut_fill_host_ex(8, 2, out.ctypes.data_as(ctypes.c_void_p)) == hog.HOG_E_INVALID
    h = ctypes.c_void_p()
    assert lib.hog_lut_build_ex(8, -1, ctypes.byref(h)) == hog.HOG_E_INVALID
    assert not h.value
    assert lib.hog_lut_orientation(None) == -1


def test_binding_leaves_one_hip_runtime_in_the_process():
    """PyTorch carries its own HIP runtime under the system one's soname.
    Loading libhog through the binding, even before anything else imports
    torch, must leave exactly one runtime mapped, so torch's device memory and
    streams belong to the runtime libhog calls."""
    code = ("import re, sys; sys.path.insert(0, %r)\n"
            "from paper_1703_06256_amd import hog\n"
            "hog.load_library()\n"
            "m = open('/proc/self/maps').read()\n"
            "print(len(set(re.findall(r'\\S*libamdhip64\\S*', m))))\n") % os.path.dirname(os.path.dirname(
                os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "1"


@pytest.mark.parametrize("orientation", [hog.HOG_ORIENT_SIGNED, hog.HOG_ORIENT_UNSIGNED])
@pytest.mark.parametrize("nb", list(range(1, 65)))
def test_soft_host_table_equals_oracle(nb, orientation):
    b0, w1 = hog.hog_lut_fill_soft_host(nb, orientation)
    ob0, ow1 = oracle.soft_table(nb, orientation == hog.HOG_ORIENT_UNSIGNED)
    assert np.array_equal(b0, ob0) and np.array_equal(w1, ow1)
