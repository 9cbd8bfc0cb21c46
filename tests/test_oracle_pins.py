"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each expected value
comes from an exact integer rule, a closed form, an invariant, a different
evaluation of the same definition (long-double angles, the literal double
sum of Eq. 5, brute-force counting against four-corner sums), or the
hand-worked fixture in tests/golden/.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import NO_BIN, ScanParams

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

DX, DY = np.meshgrid(np.arange(-255, 256), np.arange(-255, 256), indexing="xy")


def _table(n_bins):
    return oracle.bin_table(n_bins).astype(np.int64)


# --------------------------------------------------------------------------
# Sec. 2 / Fig. 2: the bin of every (dx, dy) pair.
# --------------------------------------------------------------------------
def _exact_rule_nb8(dx, dy):
    """Eight 45-degree sectors from +x, half-open, by sign tests and
    |dx|-vs-|dy| comparisons only (no trigonometry)."""
    out = np.full(dx.shape, NO_BIN, np.int64)
    conds = [
        (dx > 0) & (dy >= 0) & (dy < dx),        # [0, 45)
        (dx > 0) & (dy >= dx),                   # [45, 90)
        (dx <= 0) & (dy > -dx),                  # [90, 135)
        (dx < 0) & (dy > 0) & (dy <= -dx),       # [135, 180)
        (dx < 0) & (dy <= 0) & (dy > dx),        # [180, 225)
        (dx < 0) & (dy <= dx),                   # [225, 270)
        (dx >= 0) & (-dy > dx),                  # [270, 315)
        (dx > 0) & (dy < 0) & (-dy <= dx),       # [315, 360)
    ]
    hits = np.zeros(dx.shape, np.int64)
    for b, c in enumerate(conds):
        out[c] = b
        hits += c
    nonzero = (dx != 0) | (dy != 0)
    assert np.all(hits[nonzero] == 1) and np.all(hits[~nonzero] == 0)
    return out


def test_bins_nb8_exhaustive_exact_rule():
    assert np.array_equal(_table(8), _exact_rule_nb8(DX, DY))


def test_bins_nb4_nb2_nb1_exact_rules():
    t4 = _table(4)
    e4 = np.full(DX.shape, NO_BIN, np.int64)
    e4[(DX > 0) & (DY >= 0)] = 0
    e4[(DX <= 0) & (DY > 0)] = 1
    e4[(DX < 0) & (DY <= 0)] = 2
    e4[(DX >= 0) & (DY < 0)] = 3
    assert np.array_equal(t4, e4)
    t2 = _table(2)
    e2 = np.full(DX.shape, NO_BIN, np.int64)
    e2[(DY > 0) | ((DY == 0) & (DX > 0))] = 0
    e2[(DY < 0) | ((DY == 0) & (DX < 0))] = 1
    assert np.array_equal(t2, e2)
    t1 = _table(1)
    e1 = np.where((DX == 0) & (DY == 0), NO_BIN, 0)
    assert np.array_equal(t1, e1)


@pytest.mark.parametrize("n_bins", list(range(1, 65)))
def test_bins_on_sector_boundaries(n_bins):
    """Integer gradients hit an angle k*pi/4 exactly only on the axes and the
    diagonals (Niven: tan of a rational multiple of pi is rational only for
    0 and +-1). There the exact bin is floor(m * n_bins / 8), m = 0..7."""
    lib = oracle._load()
    dirs = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]
    for m, (ux, uy) in enumerate(dirs):
        want = (m * n_bins) // 8
        for k in (1, 2, 3, 17, 128, 254, 255):
            assert lib.orc_bin(ux * k, uy * k, n_bins) == want, (m, k, n_bins)


@pytest.mark.parametrize("n_bins", list(range(1, 65)))
def test_bins_off_boundary_match_long_double(n_bins):
    """Away from the axes and diagonals the bin must equal floor(theta n/2pi)
    evaluated in x87 long double (a different atan2 at higher precision);
    the angular margin to the nearest sector edge is far above both
    precisions, which the test also checks."""
    ld = np.longdouble
    pi = np.arctan(ld(1)) * 4
    theta = np.arctan2(DY.astype(ld), DX.astype(ld))
    theta = np.where(theta < 0, theta + 2 * pi, theta)
    pos = theta * n_bins / (2 * pi)
    tie = (DX == 0) | (DY == 0) | (np.abs(DX) == np.abs(DY))
    frac = pos - np.floor(pos)
    margin = np.minimum(frac, 1 - frac)[~tie]
    assert margin.min() > 1e-9
    want = np.floor(pos).astype(np.int64)
    got = _table(n_bins)
    assert np.array_equal(got[~tie], want[~tie])


@pytest.mark.parametrize("n_bins", list(range(1, 33)))
def test_unsigned_bins_are_signed_bins_of_twice_as_many_mod_n(n_bins):
    """Folding the angle into [0, pi) with n sectors of pi/n is the signed
    binning with 2n sectors of 2pi/(2n), taken mod n: floor(t 2n / 2pi) mod n
    = floor((t mod pi) n / pi), on the edges too. So the unsigned table is
    pinned to the signed one, itself pinned above."""
    u = oracle.bin_table(n_bins, unsigned=True).astype(np.int64)
    s2 = oracle.bin_table(2 * n_bins).astype(np.int64)
    want = np.where(s2 == NO_BIN, NO_BIN, s2 % n_bins)
    assert np.array_equal(u, want)


@pytest.mark.parametrize("n_bins", [9, 33, 47, 64])
def test_unsigned_bins_off_edges_match_long_double(n_bins):
    """n > 32 has no signed table of 2n bins to compare with: off the axes and
    diagonals the unsigned bin must equal floor((theta mod pi) n / pi) in x87
    long double, with a margin to the edges far above both precisions."""
    ld = np.longdouble
    pi = np.arctan(ld(1)) * 4
    theta = np.arctan2(DY.astype(ld), DX.astype(ld))
    theta = np.where(theta < 0, theta + pi, theta)
    pos = theta * n_bins / pi
    tie = (DX == 0) | (DY == 0) | (np.abs(DX) == np.abs(DY))
    frac = pos - np.floor(pos)
    assert np.minimum(frac, 1 - frac)[~tie].min() > 1e-9
    got = oracle.bin_table(n_bins, unsigned=True)
    assert np.array_equal(got[~tie], np.floor(pos).astype(np.int64)[~tie])
    # axes and diagonals: (m mod 4) n / 4 for the direction m pi / 4
    for (dx, dy), m in [((7, 0), 0), ((-7, 0), 0), ((0, 7), 2), ((0, -7), 2), ((7, 7), 1),
                        ((-7, -7), 1), ((-7, 7), 3), ((7, -7), 3)]:
        assert oracle.bin_of(dx, dy, n_bins, unsigned=True) == (m * n_bins) // 4


def test_unsigned_bins_opposite_gradients_share_a_bin_and_9_bin_examples():
    u = oracle.bin_table(9, unsigned=True)
    assert np.array_equal(u, u[::-1, ::-1])  # (dx, dy) and (-dx, -dy)
    # 9 bins of 20 degrees over 0..180
    cases = {(1, 0): 0, (-1, 0): 0, (0, 1): 4, (0, -1): 4, (1, 1): 2, (-1, -1): 2, (-1, 1): 6,
             (1, -1): 6, (5, -3): 7, (-5, 3): 7, (10, 1): 0, (1, 10): 4, (-10, 1): 8}
    for (dx, dy), want in cases.items():
        assert oracle.bin_of(dx, dy, 9, unsigned=True) == want, (dx, dy)


def test_unsigned_bin_map_is_signed_map_of_twice_the_bins_mod_n():
    """Through the whole bin map (Eq. 1, channel choice, border): unsigned
    with n bins equals signed with 2n bins mod n; an inverted image (every
    gradient negated) has the same unsigned map."""
    rng = np.random.default_rng(77)
    img = rng.integers(0, 256, (37, 53, 3)).astype(np.uint8)
    for n in (4, 9, 16):
        u = oracle.bin_map(img, n, unsigned=True).astype(np.int64)
        s2 = oracle.bin_map(img, 2 * n).astype(np.int64)
        assert np.array_equal(u, np.where(s2 == NO_BIN, NO_BIN, s2 % n))
        assert np.array_equal(u, oracle.bin_map(255 - img, n, unsigned=True))


@pytest.mark.parametrize("n_bins", [8, 18])
def test_bins_reflection(n_bins):
    """Mirroring dy mirrors the angle: bin(dx,-dy) = n-1-bin(dx,dy) off edges."""
    t = _table(n_bins)
    flipped = t[::-1, :]  # row index dy+255 -> -dy+255
    tie = (DY == 0) | (DX == 0) | (np.abs(DX) == np.abs(DY))
    ok = ~tie
    assert np.array_equal(flipped[ok], n_bins - 1 - t[ok])


# --------------------------------------------------------------------------
# Eq. 1: the stencil, border and colour rule.
# --------------------------------------------------------------------------
def _ramp(w, h, a, b, c0=100):
    x = np.arange(w)[None, :]
    y = np.arange(h)[:, None]
    return (c0 + a * x + b * y).astype(np.uint8)


@pytest.mark.parametrize("a,b,want", [
    (1, 0, 0), (1, 1, 1), (0, 1, 2), (-1, 1, 3),
    (-1, 0, 4), (-1, -1, 5), (0, -1, 6), (1, -1, 7), (2, 1, 0), (1, 3, 1),
])
def test_ramp_gives_one_bin(a, b, want):
    """P = c + a x + b y has dx = 2a, dy = 2b at every interior pixel."""
    img = _ramp(12, 10, a, b)
    m = oracle.bin_map(img, 8)
    assert np.all(m[1:-1, 1:-1] == want)
    assert np.all(m[0, :] == NO_BIN) and np.all(m[-1, :] == NO_BIN)
    assert np.all(m[:, 0] == NO_BIN) and np.all(m[:, -1] == NO_BIN)


def test_flat_and_tiny_images_have_no_bins():
    assert np.all(oracle.bin_map(np.full((9, 7), 77, np.uint8), 8) == NO_BIN)
    for w, h in [(1, 1), (2, 5), (5, 2), (2, 2)]:
        img = np.random.default_rng(0).integers(0, 256, (h, w), dtype=np.uint8)
        assert np.all(oracle.bin_map(img, 8) == NO_BIN)


def test_colour_channel_with_largest_gradient_wins_ties_to_lowest():
    w, h = 10, 8
    img = np.zeros((h, w, 3), np.uint8)
    img[:, :, 0] = _ramp(w, h, 1, 0)    # (2, 0): magnitude 4, bin 0
    img[:, :, 1] = _ramp(w, h, 0, 2)    # (0, 4): magnitude 16, bin 2
    img[:, :, 2] = _ramp(w, h, -2, 0, 200)  # (-4, 0): magnitude 16, bin 4
    m = oracle.bin_map(img, 8)
    assert np.all(m[1:-1, 1:-1] == 2)  # channel 1 beats 0, ties channel 2
    img[:, :, 2] = _ramp(w, h, -3, 0, 200)  # (-6, 0): magnitude 36 wins
    assert np.all(oracle.bin_map(img, 8)[1:-1, 1:-1] == 4)


def _read_golden(name):
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                sections[cur] = []
            else:
                sections[cur].append([int(v) for v in line.split()])
    return {k: np.array(v, dtype=np.int64) for k, v in sections.items()}


def test_golden_hand_worked_5x5():
    g = _read_golden("gray5x5.txt")
    img = g["image"].astype(np.uint8)
    assert np.array_equal(oracle.bin_map(img, 8), g["bins nb=8"])
    assert np.array_equal(oracle.bin_map(img, 4), g["bins nb=4"])
    planes = oracle.integral(oracle.bin_map(img, 8), 8)
    assert np.array_equal(planes[1], g["plane nb=8 bin=1"])
    assert np.array_equal(planes[6], g["plane nb=8 bin=6"])


# --------------------------------------------------------------------------
# Eq. 4 / Eq. 5: integral images.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("w,h", [(1, 1), (1, 7), (7, 1), (5, 5), (16, 16), (13, 9)])
def test_integral_recurrence_equals_literal_sum(w, h):
    rng = np.random.default_rng(w * 100 + h)
    bins = rng.integers(0, 6, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < 0.2] = NO_BIN
    assert np.array_equal(oracle.integral(bins, 6), oracle.integral_literal(bins, 6))


def test_integral_closed_form_single_bin():
    w, h = 23, 17
    bins = np.full((h, w), 3, np.uint8)
    p = oracle.integral(bins, 5)
    x = np.arange(w + 1)[None, :]
    y = np.arange(h + 1)[:, None]
    assert np.array_equal(p[3], (x * y).astype(np.uint32))  # ii(x,y) = (x+1)(y+1)
    for b in (0, 1, 2, 4):
        assert not p[b].any()


def test_integral_invariants():
    rng = np.random.default_rng(7)
    h, w, nb = 41, 67, 9
    bins = rng.integers(0, nb, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < 0.15] = NO_BIN
    p = oracle.integral(bins, nb).astype(np.int64)
    # corner: the planes sum to the number of binned pixels
    assert p[:, h, w].sum() == np.count_nonzero(bins != NO_BIN)
    # four-point differencing recovers the one-hot decomposition of Eq. 4
    d = p[:, 1:, 1:] - p[:, :-1, 1:] - p[:, 1:, :-1] + p[:, :-1, :-1]
    onehot = (bins[None, :, :] == np.arange(nb)[:, None, None]).astype(np.int64)
    assert np.array_equal(d, onehot)
    # guard row/column and monotonicity
    assert not p[:, 0, :].any() and not p[:, :, 0].any()
    assert np.all(np.diff(p, axis=1) >= 0) and np.all(np.diff(p, axis=2) >= 0)


@pytest.mark.parametrize("bits", [16, 8])
def test_narrow_integral_closed_form_wraps(bits):
    """One bin everywhere: ii(x, y) = (x + 1)(y + 1), so the narrow planes
    hold that product mod 2^bits -- here it wraps (up to 400 x 300 pixels)."""
    w, h = 400, 300
    bins = np.full((h, w), 2, np.uint8)
    p = oracle.integral_mod(bins, 3, bits)
    assert p.dtype == (np.uint16 if bits == 16 else np.uint8)
    x = np.arange(w + 1, dtype=np.int64)[None, :]
    y = np.arange(h + 1, dtype=np.int64)[:, None]
    assert np.array_equal(p[2].astype(np.int64), (x * y) % (1 << bits))
    assert int((x * y).max()) >= 1 << bits  # the case does wrap
    assert not p[0].any() and not p[1].any()


@pytest.mark.parametrize("bits", [16, 8])
def test_narrow_integral_four_corners_count_small_rectangles(bits):
    """The reading behind narrow planes: on the planes mod 2^bits, the
    four-corner sum of Eq. 6 taken mod 2^bits equals the brute-force count of
    any rectangle with fewer than 2^bits pixels, wherever it lies (values far
    beyond 2^bits below and left of it); at exactly 2^bits pixels of one bin
    it reads 0, so the bound is tight."""
    rng = np.random.default_rng(100 + bits)
    h, w, nb = 700, 500, 3  # 350,000 pixels: every plane wraps mod 2^16 and 2^8
    bins = rng.integers(0, nb, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < 0.05] = NO_BIN
    p = oracle.integral_mod(bins, nb, bits).astype(np.int64)
    m = 1 << bits
    for _ in range(300):
        rh = int(rng.integers(1, min(h, m - 1) + 1))
        rw = int(rng.integers(1, min(w, (m - 1) // rh) + 1))
        y0 = int(rng.integers(0, h - rh + 1))
        x0 = int(rng.integers(0, w - rw + 1))
        y1, x1 = y0 + rh, x0 + rw
        assert rh * rw < m
        four = (p[:, y1, x1] + p[:, y0, x0] - p[:, y0, x1] - p[:, y1, x0]) % m
        brute = [(bins[y0:y1, x0:x1] == n).sum() for n in range(nb)]
        assert list(four) == brute
    # tightness: 2^bits pixels, all of bin 0
    side = 1 << (bits // 2)
    one = np.zeros((side + 3, side + 5), np.uint8)
    q = oracle.integral_mod(one, 1, bits).astype(np.int64)
    y0, x0 = 2, 3
    four = (q[0, y0 + side, x0 + side] + q[0, y0, x0] - q[0, y0, x0 + side] - q[0, y0 + side, x0]) % m
    assert four == 0


# --------------------------------------------------------------------------
# Eq. 3 / Eq. 6: area histograms.
# --------------------------------------------------------------------------
def test_cell_hist_equals_four_corner_sums():
    """Brute-force counts equal ii(4) + ii(1) - ii(2) - ii(3) on the planes."""
    rng = np.random.default_rng(11)
    h, w, nb = 53, 70, 8
    bins = rng.integers(0, nb, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < 0.3] = NO_BIN
    p = oracle.integral(bins, nb).astype(np.int64)
    ch = oracle.cell_hist(bins, nb, 8).astype(np.int64)
    hc, wc = h // 8, w // 8
    assert ch.shape == (hc, wc, nb)
    ys = np.arange(hc + 1) * 8
    xs = np.arange(wc + 1) * 8
    c = p[:, ys][:, :, xs]  # corners on the padded grid
    four = c[:, 1:, 1:] + c[:, :-1, :-1] - c[:, :-1, 1:] - c[:, 1:, :-1]
    assert np.array_equal(four.transpose(1, 2, 0), ch)
    assert np.all(ch.sum(axis=2) <= 64)


def test_cell_hist_ramp_values():
    """A ramp bins every interior pixel into one bin; a border-touching cell
    loses its border row/column: interior 64, edge 56, corner 49."""
    img = _ramp(32, 24, 1, 0)
    ch = oracle.cell_hist(oracle.bin_map(img, 8), 8, 8)
    tot = ch.sum(axis=2)
    assert np.all(ch[:, :, 1:] == 0)
    want = np.array([[49, 56, 56, 49], [56, 64, 64, 56], [49, 56, 56, 49]])
    assert np.array_equal(tot, want)


# --------------------------------------------------------------------------
# Sec. 3.1 / Fig. 4 and Sec. 4: features and scores.
# --------------------------------------------------------------------------
def _bins_random(h, w, nb, seed, empty=0.2):
    rng = np.random.default_rng(seed)
    bins = rng.integers(0, nb, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < empty] = NO_BIN
    return bins


def test_raw_feature_is_cell_histograms_in_order():
    nb = 8
    bins = _bins_random(150, 90, nb, 3)
    ch = oracle.cell_hist(bins, nb, 8)
    p = ScanParams(norm=0)
    for wx, wy in [(0, 0), (3, 1), (3, 2)]:
        f = oracle.window_feature(bins, nb, p, wx, wy)
        want = ch[wy:wy + 16, wx:wx + 8, :].reshape(-1)
        assert np.array_equal(f, want.astype(np.float64))


def test_l2_feature_closed_form():
    nb = 8
    bins = _bins_random(140, 80, nb, 5)
    ch = oracle.cell_hist(bins, nb, 8).astype(np.float64)
    p = ScanParams(norm=1, eps=1e-3)
    f = oracle.window_feature(bins, nb, p, 1, 1)
    assert f.shape == (7 * 15 * 4 * nb,)
    fb = f.reshape(15, 7, 4, nb)
    for by in range(15):
        for bx in range(7):
            cells = ch[1 + by:1 + by + 2, 1 + bx:1 + bx + 2, :]  # [v][u][n]
            v = cells.reshape(4, nb)
            nv = np.sqrt((v ** 2).sum())
            assert np.allclose(fb[by, bx], v / np.sqrt(nv ** 2 + 1e-6), rtol=1e-14, atol=0)
            # |f| = |v| / sqrt(|v|^2 + eps^2)
            assert abs(np.linalg.norm(fb[by, bx]) - nv / np.sqrt(nv ** 2 + 1e-6)) < 1e-14


def test_l2_feature_empty_block_and_uniform_block():
    nb = 8
    bins = np.full((128, 64), NO_BIN, np.uint8)
    p = ScanParams(norm=1)
    assert not oracle.window_feature(bins, nb, p, 0, 0).any()
    bins = np.full((128, 64), 2, np.uint8)  # every cell 64 in bin 2
    f = oracle.window_feature(bins, nb, p, 0, 0).reshape(105, 4, nb)
    want = 64.0 / np.sqrt(4 * 64.0 ** 2 + 1e-6)
    assert np.allclose(f[:, :, 2], want, rtol=1e-15)
    assert not np.delete(f, 2, axis=2).any()


def test_scores_closed_forms():
    nb = 8
    bins = _bins_random(140, 80, nb, 9)
    p = ScanParams(norm=0)
    dim = p.dim(nb)
    ones = np.ones((1, dim), np.float32)
    s, a, _, wxs, wys = oracle.score_windows(bins, nb, p, ones, np.array([0.5], np.float32))
    # all-ones template on raw features counts the window's binned pixels
    for i in range(len(wxs)):
        x0, y0 = wxs[i] * 8, wys[i] * 8
        n = np.count_nonzero(bins[y0:y0 + 128, x0:x0 + 64] != NO_BIN)
        assert s[i, 0] == n + 0.5 and a[i, 0] == n + 0.5
    # one-hot templates select single features; linearity in the template
    rng = np.random.default_rng(1)
    t = np.zeros((3, dim), np.float32)
    t[0, 17] = 1.0
    t[1] = rng.standard_normal(dim).astype(np.float32)
    t[2] = 2 * t[1] - t[0]
    s, _, f, _, _ = oracle.score_windows(bins, nb, p, t, np.zeros(3, np.float32),
                                         want_feats=True)
    assert np.array_equal(s[:, 0], f[:, 17])
    assert np.allclose(s[:, 2], 2 * s[:, 1] - s[:, 0], rtol=1e-12, atol=1e-9)


def test_scores_flat_image_equal_bias():
    img = np.full((140, 80, 3), 90, np.uint8)
    bins = oracle.bin_map(img, 8)
    for norm in (0, 1):
        p = ScanParams(norm=norm)
        t = np.random.default_rng(2).standard_normal((2, p.dim(8))).astype(np.float32)
        s, _, _, _, _ = oracle.score_windows(bins, 8, p, t, np.array([0.25, -1.5], np.float32))
        assert np.all(s[:, 0] == 0.25) and np.all(s[:, 1] == -1.5)


def test_window_grid():
    p = ScanParams()
    assert oracle.window_grid(320, 240, p) == (33, 15)
    assert oracle.window_grid(800, 600, p) == (93, 60)
    assert oracle.window_grid(63, 500, p) == (0, 0)
    assert oracle.window_grid(64, 128, p) == (1, 1)
    assert p.dim(8) == 1024 and ScanParams(norm=1).dim(8) == 3360
    assert ScanParams(norm=1).dim(18) == 7560


# --------------------------------------------------------------------------
# Image pyramid (nearest neighbour).
# --------------------------------------------------------------------------
def test_pyramid_levels_1920x1080():
    lv = oracle.pyramid(1920, 1080, 1.05, 64, 128)
    assert len(lv) == 44
    assert lv[0] == (1920, 1080, 1.0)
    assert lv[1][:2] == (1828, 1028)
    assert lv[-1][:2] == (235, 132)
    assert sum(w * h for w, h, _ in lv) == 21970720
    for l, (w, h, s) in enumerate(lv):
        assert abs(s - 1.05 ** l) < 1e-12 * 1.05 ** l
        assert w == int(np.floor(1920 / s)) and h == int(np.floor(1080 / s))


def test_pyramid_single_level_and_limits():
    assert oracle.pyramid(3, 3, 1.0, 64, 128, 1) == [(3, 3, 1.0)]
    assert len(oracle.pyramid(800, 600, 1.1, 64, 128, 3)) == 3


def test_resize_nn_closed_forms():
    rng = np.random.default_rng(4)
    img = rng.integers(0, 256, (40, 60, 3), dtype=np.uint8)
    assert np.array_equal(oracle.resize_nn(img, 1.0, 60, 40), img)
    assert np.array_equal(oracle.resize_nn(img, 2.0, 30, 20), img[::2, ::2])
    out = oracle.resize_nn(img, 1.5, 40, 26)
    assert np.array_equal(out[5, 7], img[7, 10])  # floor(5*1.5)=7, floor(7*1.5)=10


# --------------------------------------------------------------------------
# Soft votes (Sec. 2's two-bin split, quantised).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_bins,unsigned", [(1, False), (4, False), (8, False), (9, True), (18, False),
                                             (18, True), (64, False)])
def test_soft_vote_centre_of_mass_is_the_angle(n_bins, unsigned):
    """Independent of the oracle's arithmetic: the two shares sum to one
    pixel, and their centre of mass (b0 + 1/2 + w1/Q bin widths) is the
    gradient's angle, within the quantisation (half a unit) -- checked
    against x87 long double atan2 over the whole table."""
    q = oracle.SOFT_Q
    b0, w1 = oracle.soft_table(n_bins, unsigned)
    zero = (DX == 0) & (DY == 0)
    assert np.all(b0[zero] == NO_BIN) and np.all(w1[zero] == 0)
    assert np.all(b0[~zero] < n_bins) and np.all(w1[~zero] <= q)
    ld = np.longdouble
    pi = np.arctan(ld(1)) * 4
    rng_ = pi if unsigned else 2 * pi
    t = np.arctan2(DY.astype(ld), DX.astype(ld))
    t = np.where(t < 0, t + rng_, t)
    width = rng_ / n_bins
    centre = (b0.astype(ld) + ld(0.5) + w1.astype(ld) / q) * width
    d = np.mod(centre - t + rng_ / 2, rng_) - rng_ / 2  # signed difference mod the range
    assert np.abs(d[~zero]).max() <= width / (2 * q) + ld(1e-12)


def test_soft_vote_axes_and_centres():
    # a gradient on a bin centre gives all of its vote to that bin
    assert oracle.soft_vote(1, 1, 4) == (0, 0)            # 45 deg, centre of bin 0 of 4
    assert oracle.soft_vote(-1, 1, 4) == (1, 0)
    # on a sector edge it is split evenly
    assert oracle.soft_vote(1, 0, 8) == (7, 16)            # 0 deg: between bins 7 and 0
    assert oracle.soft_vote(0, 1, 4) == (0, 16)            # 90 deg: between bins 0 and 1
    # 90 of 180 degrees with 9 bins of 20: the centre of bin 4, whole vote there
    assert oracle.soft_vote(0, 5, 9, unsigned=True) == (4, 0)
    assert oracle.soft_vote(0, -5, 9, unsigned=True) == (4, 0)
    # 0 degrees unsigned: between the last bin and bin 0
    assert oracle.soft_vote(-3, 0, 9, unsigned=True) == (8, 16)
    assert oracle.soft_vote(0, 0, 8) == (NO_BIN, 0)


def test_soft_integral_closed_form_and_invariants():
    q = oracle.SOFT_Q
    h, w, nb = 13, 21, 5
    b0 = np.full((h, w), 3, np.uint8)
    w1 = np.full((h, w), 10, np.uint8)
    p = oracle.soft_integral(b0, w1, nb).astype(np.int64)
    x = np.arange(w + 1)[None, :]
    y = np.arange(h + 1)[:, None]
    assert np.array_equal(p[3], (q - 10) * x * y) and np.array_equal(p[4], 10 * x * y)
    assert not p[[0, 1, 2]].any()
    rng = np.random.default_rng(5)
    b0 = rng.integers(0, nb, (h, w)).astype(np.uint8)
    w1 = rng.integers(0, q + 1, (h, w)).astype(np.uint8)
    b0[rng.random((h, w)) < 0.2] = NO_BIN
    p = oracle.soft_integral(b0, w1, nb).astype(np.int64)
    assert p[:, h, w].sum() == q * np.count_nonzero(b0 != NO_BIN)
    d = p[:, 1:, 1:] - p[:, :-1, 1:] - p[:, 1:, :-1] + p[:, :-1, :-1]  # per-pixel votes
    for n in range(nb):
        want = np.where(b0 == n, q - w1.astype(np.int64), 0) + np.where((b0 + 1) % nb == n, w1, 0)
        want = np.where(b0 == NO_BIN, 0, want)
        assert np.array_equal(d[n], want)


def test_soft_cell_hist_equals_four_corners_and_centred_votes_equal_hard_counts():
    rng = np.random.default_rng(9)
    h, w, nb = 48, 72, 7
    b0 = rng.integers(0, nb, (h, w)).astype(np.uint8)
    w1 = rng.integers(0, oracle.SOFT_Q + 1, (h, w)).astype(np.uint8)
    b0[rng.random((h, w)) < 0.1] = NO_BIN
    p = oracle.soft_integral(b0, w1, nb).astype(np.int64)
    ch = oracle.soft_cell_hist(b0, w1, nb, 8).astype(np.int64)
    c = p[:, ::8][:, :, ::8]
    four = c[:, 1:, 1:] + c[:, :-1, :-1] - c[:, :-1, 1:] - c[:, 1:, :-1]
    assert np.array_equal(four.transpose(1, 2, 0), ch)
    # a diagonal ramp puts every interior gradient on the 45-degree centre of bin 0 of 4
    yy, xx = np.mgrid[0:40, 0:48]
    img = (2 * xx + 2 * yy).astype(np.uint8)
    sb0, sw1 = oracle.soft_bin_map(img, 4)
    hard = oracle.bin_map(img, 4)
    assert np.array_equal(oracle.soft_cell_hist(sb0, sw1, 4, 8),
                          oracle.SOFT_Q * oracle.cell_hist(hard, 4, 8))


@pytest.mark.parametrize("norm,cell,wcx,wcy", [(0, 8, 8, 16), (1, 8, 8, 16), (1, 6, 5, 7), (0, 4, 3, 9)])
def test_features_from_cells_equal_the_brute_force_window_feature(norm, cell, wcx, wcy):
    """The numpy feature builder the soft-vote scores use, fed hard cell
    counts, equals the C oracle's brute-force window feature (pinned above)
    element for element; and soft votes that all sit on bin centres (a
    diagonal ramp, 4 bins) give Q times the hard counts, hence the same
    features once divided by Q."""
    p = ScanParams(cell=cell, win_cells_x=wcx, win_cells_y=wcy, norm=norm)
    rng = np.random.default_rng(norm * 10 + cell)
    h, w, nb = 140, 90, 6
    bins = rng.integers(0, nb, (h, w)).astype(np.uint8)
    bins[rng.random((h, w)) < 0.2] = NO_BIN
    cells = oracle.cell_hist(bins, nb, cell)
    mx, my = (w // cell) - wcx, (h // cell) - wcy
    for wx, wy in [(0, 0), (min(1, mx), min(2, my)), (mx, my)]:
        assert np.allclose(oracle.features_from_cells(cells, p, wx, wy),
                           oracle.window_feature(bins, nb, p, wx, wy), rtol=1e-14, atol=0)
    yy, xx = np.mgrid[0:140, 0:90]
    img = (2 * xx + 2 * yy).astype(np.uint8)
    sb0, sw1 = oracle.soft_bin_map(img, 4)
    soft_cells = oracle.soft_cell_hist(sb0, sw1, 4, cell) / oracle.SOFT_Q
    assert np.allclose(oracle.features_from_cells(soft_cells, p, 1, 1),
                       oracle.window_feature(oracle.bin_map(img, 4), 4, p, 1, 1), rtol=1e-14, atol=0)
