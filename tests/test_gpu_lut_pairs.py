"""Sec. 2's lookup table on the device, over every (dx, dy) in [-255, 255]^2.

- The device copies a hog_lut holds (the full table, the dy >= 0 half that the
  bin-map kernel stages in LDS with its mirror flags, and the soft-vote table)
  are read back from device memory and compared with the oracle's FP64
  tables.
- The bin-map kernel itself is fed an image that realises every gradient
  pair: lattice pixel (3 i + 1, 3 j + 1) has left/right neighbours max(0, -dx)
  and max(0, -dx) + dx, up/down neighbours max(0, -dy) and max(0, -dy) + dy,
  with dx = i - 255 and dy = j - 255. The neighbour sets of lattice pixels
  are disjoint at spacing 3, so one 1533 x 1533 image covers all 261,121
  pairs; the other pixels are seeded noise. With 3 channels the pattern sits
  in channel (i + j) mod 3 and the other two are flat, so the channel choice
  (largest dx^2 + dy^2, Eq. 1 per channel) is exercised as well. Every pixel
  of the bin map is compared with the oracle (hard votes: bins; soft votes:
  the (b0, w1) pairs).
"""
import numpy as np
import pytest

import oracle
from paper_1703_06256_amd import hog

BINS = (1, 2, 8, 9, 18, 20, 36, 64)
ORIENT = (hog.HOG_ORIENT_SIGNED, hog.HOG_ORIENT_UNSIGNED)
SIDE = 3 * 511


def pair_image(channels: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    img = np.empty((SIDE, SIDE, channels), np.uint8)
    img[:] = 128  # flat channels
    j, i = np.mgrid[0:511, 0:511]
    dx, dy = i - 255, j - 255
    x, y = 3 * i + 1, 3 * j + 1
    ch = (i + j) % channels
    pat = rng.integers(0, 256, (SIDE, SIDE), dtype=np.uint8)
    left = np.maximum(0, -dx)
    up = np.maximum(0, -dy)
    pat[y, x - 1] = left
    pat[y, x + 1] = left + dx
    pat[y - 1, x] = up
    pat[y + 1, x] = up + dy
    # The pattern channel of each 3 x 3 lattice cell holds pat; the others stay flat.
    cell_ch = np.repeat(np.repeat(ch, 3, axis=0), 3, axis=1)
    for c in range(channels):
        img[:, :, c] = np.where(cell_ch == c, pat, img[:, :, c])
    return img


def lattice_pairs(img: np.ndarray):
    """(dx, dy) of every lattice pixel, read from the image itself."""
    j, i = np.mgrid[0:511, 0:511]
    x, y = 3 * i + 1, 3 * j + 1
    ch = (i + j) % img.shape[2]
    p = img.astype(np.int32)
    dx = p[y, x + 1, ch] - p[y, x - 1, ch]
    dy = p[y + 1, x, ch] - p[y - 1, x, ch]
    return dx, dy


@pytest.mark.parametrize("channels", [1, 3])
def test_pair_image_covers_every_gradient(channels):
    """The construction itself (CPU): every pair appears at exactly one
    lattice pixel."""
    img = pair_image(channels, 77 + channels)
    dx, dy = lattice_pairs(img)
    keys = (dy + 255) * 511 + (dx + 255)
    assert np.unique(keys).size == 511 * 511
    assert np.array_equal(np.sort(keys.reshape(-1)), np.arange(511 * 511))


@pytest.mark.gpu
@pytest.mark.parametrize("orientation", ORIENT)
@pytest.mark.parametrize("nb", BINS)
def test_device_tables_equal_oracle(nb, orientation):
    unsigned = orientation == hog.HOG_ORIENT_UNSIGNED
    lut = hog.hog_lut_build(nb, orientation)
    full = lut.device_table(hog.HOG_LUT_DEVICE_FULL)
    want = oracle.bin_table(nb, unsigned)
    assert np.array_equal(full, want)
    # dy >= 0 rows: the bin in the low 6 bits, and the flag that gives the
    # mirrored entry: bin(dx, -dy) = nb - 1 - bin(dx, dy) + f.
    half = lut.device_table(hog.HOG_LUT_DEVICE_HALF)
    up = want[255:, :]
    dn = want[255::-1, :]
    nob = up == hog.HOG_NO_BIN
    assert np.array_equal(nob, half == hog.HOG_NO_BIN)
    assert np.array_equal(half[~nob] & 63, up[~nob])
    f = (half.astype(np.int32) >> 6) & 1
    assert np.all(half[~nob] >> 7 == 0)
    rows = np.arange(256)[:, None] > 0
    m = ~nob & rows
    assert np.array_equal(dn[m].astype(np.int32), nb - 1 - up[m].astype(np.int32) + f[m])
    soft = lut.device_table(hog.HOG_LUT_DEVICE_SOFT)
    b0, w1 = oracle.soft_table(nb, unsigned)
    assert np.array_equal(soft & 255, b0) and np.array_equal(soft >> 8, w1)
    lut.free()


def _bin_map_gpu(img, nb, orientation, votes, lut_global=0):
    import torch
    c = img.shape[2]
    desc = hog.make_desc(SIDE, SIDE, channels=c, n_bins=nb, votes=votes)
    plan = hog.Plan(desc)
    if lut_global:
        t = hog.plan_tiles(plan)
        hog.set_plan_tiles(plan, t.bin_chunk, t.score_rows, 1, lut_global=1)
        assert hog.plan_tiles(plan).lut_global == 1
    lut = hog.hog_lut_build(nb, orientation)
    img_t = torch.from_numpy(np.ascontiguousarray(img).reshape(-1)).cuda()
    bins = torch.empty(plan.sizes.bins_bytes, dtype=torch.uint8, device="cuda")
    hog.hog_bin_map(plan, lut, img_t, bins)
    torch.cuda.synchronize()
    out = hog.level_bins(plan, bins.cpu().numpy(), 0)
    lut.free()
    plan.destroy()
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("lut_global", [0, 1])
@pytest.mark.parametrize("channels", [1, 3])
@pytest.mark.parametrize("orientation", ORIENT)
@pytest.mark.parametrize("nb", BINS)
def test_bin_map_every_gradient_pair(nb, orientation, channels, lut_global):
    """Both table placements: the LDS half table with its mirror flags, and
    the full table read through L2 (hog_tiles.lut_global)."""
    unsigned = orientation == hog.HOG_ORIENT_UNSIGNED
    img = pair_image(channels, 500 + nb + 7 * channels + orientation)
    got = _bin_map_gpu(img, nb, orientation, hog.HOG_VOTES_HARD, lut_global)
    want = oracle.bin_map(img, nb, unsigned)
    assert np.array_equal(got, want)
    # Every table entry was looked up at some lattice pixel.
    dx, dy = lattice_pairs(img)
    lat = got[1::3, 1::3]
    assert np.array_equal(lat, oracle.bin_table(nb, unsigned)[dy + 255, dx + 255])


@pytest.mark.gpu
@pytest.mark.parametrize("channels", [1, 3])
@pytest.mark.parametrize("orientation", ORIENT)
@pytest.mark.parametrize("nb", BINS)
def test_soft_bin_map_every_gradient_pair(nb, orientation, channels):
    unsigned = orientation == hog.HOG_ORIENT_UNSIGNED
    img = pair_image(channels, 900 + nb + 7 * channels + orientation)
    gb0, gw1 = _bin_map_gpu(img, nb, orientation, hog.HOG_VOTES_SOFT)
    b0, w1 = oracle.soft_bin_map(img, nb, unsigned)
    assert np.array_equal(gb0, b0) and np.array_equal(gw1, w1)
    dx, dy = lattice_pairs(img)
    tb0, tw1 = oracle.soft_table(nb, unsigned)
    assert np.array_equal(gb0[1::3, 1::3], tb0[dy + 255, dx + 255])
    assert np.array_equal(gw1[1::3, 1::3], tw1[dy + 255, dx + 255])
