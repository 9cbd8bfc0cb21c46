"""CPU oracle for the fast-HOG hot path -- test infrastructure only.

A thin ctypes wrapper over ``oracle.c`` (plain C, FP64, brute force; see
that file's header for what each function follows in the paper). Only the
test suite, the smoke check and the benchmark's CPU-baseline leg import
this package. It never imports the product package and the product never
imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

NO_BIN = 255
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, one thread)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        p = ctypes.c_void_p
        lib.orc_bin.argtypes = [i32, i32, i32]
        lib.orc_bin.restype = i32
        lib.orc_bin_table.argtypes = [i32, p]
        lib.orc_bin_table.restype = i32
        lib.orc_bin_map.argtypes = [p, i32, i32, i32, i64, i32, p]
        lib.orc_bin_unsigned.argtypes = [i32, i32, i32]
        lib.orc_bin_unsigned.restype = i32
        lib.orc_bin_table_ex.argtypes = [i32, i32, p]
        lib.orc_bin_table_ex.restype = i32
        lib.orc_bin_map_ex.argtypes = [p, i32, i32, i32, i64, i32, i32, p]
        lib.orc_bin_map_ex.restype = i32
        lib.orc_soft_vote.argtypes = [i32, i32, i32, i32, p, p]
        lib.orc_soft_vote.restype = i32
        lib.orc_soft_table.argtypes = [i32, i32, p, p]
        lib.orc_soft_table.restype = i32
        lib.orc_soft_bin_map.argtypes = [p, i32, i32, i32, i64, i32, i32, p, p]
        lib.orc_soft_bin_map.restype = i32
        lib.orc_soft_integral.argtypes = [p, p, i32, i32, i32, p]
        lib.orc_soft_integral.restype = i32
        lib.orc_soft_cell_hist.argtypes = [p, p, i32, i32, i32, i32, p]
        lib.orc_soft_cell_hist.restype = i32
        lib.orc_pyramid.argtypes = [i32, i32, dbl, i32, i32, i32, i32, p, p, p]
        lib.orc_resize_nn.argtypes = [p, i32, i32, i32, i64, dbl, i32, i32, p]
        lib.orc_integral.argtypes = [p, i32, i32, i32, p]
        lib.orc_integral_literal.argtypes = [p, i32, i32, i32, p]
        lib.orc_cell_hist.argtypes = [p, i32, i32, i32, i32, p]
        lib.orc_feature_dim.argtypes = [i32, i32, i32, i32, i32]
        lib.orc_window_feature.argtypes = [p, i32, i32, i32, i32, i32, i32, i32, i32, dbl,
                                           i32, i32, p]
        lib.orc_window_grid.argtypes = [i32, i32, i32, i32, i32, p, p]
        lib.orc_score_windows.argtypes = [p, i32, i32, i32, i32, i32, i32, i32, i32, dbl,
                                          p, p, i32, i32, p, p, p, p, p]
        for name in ("orc_bin_map", "orc_pyramid", "orc_resize_nn", "orc_integral",
                     "orc_integral_literal", "orc_cell_hist", "orc_feature_dim",
                     "orc_window_feature", "orc_window_grid", "orc_score_windows"):
            getattr(lib, name).restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


# --------------------------------------------------------------------------
def bin_of(dx: int, dy: int, n_bins: int, unsigned: bool = False) -> int:
    """Orientation bin of one gradient (FP64 atan2; 255 for a zero gradient);
    unsigned: the angle mod pi."""
    fn = _load().orc_bin_unsigned if unsigned else _load().orc_bin
    r = fn(int(dx), int(dy), int(n_bins))
    _check(r, "bin")
    return r


def bin_table(n_bins: int, unsigned: bool = False) -> np.ndarray:
    """bin_of over every (dx, dy) in [-255, 255]^2, as uint8[dy+255][dx+255]."""
    out = np.empty((511, 511), dtype=np.uint8)
    _check(_load().orc_bin_table_ex(int(n_bins), int(unsigned), _ptr(out)), "bin_table")
    return out


def bin_map(img: np.ndarray, n_bins: int, unsigned: bool = False) -> np.ndarray:
    """Bin map (uint8, h x w) of an image of shape (h, w) or (h, w, c)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        img = img[:, :, None]
    h, w, c = img.shape
    out = np.empty((h, w), dtype=np.uint8)
    _check(_load().orc_bin_map_ex(_ptr(img), w, h, c, w * c, n_bins, int(unsigned), _ptr(out)),
           "bin_map")
    return out


SOFT_Q = 32  # vote units per pixel (soft votes)


def soft_vote(dx: int, dy: int, n_bins: int, unsigned: bool = False):
    """(b0, w1) of one gradient: w1 units to bin b0 + 1 mod n, SOFT_Q - w1 to
    b0; (255, 0) for a zero gradient."""
    b0, w1 = ctypes.c_int(), ctypes.c_int()
    _check(_load().orc_soft_vote(int(dx), int(dy), int(n_bins), int(unsigned), ctypes.byref(b0),
                                 ctypes.byref(w1)), "soft_vote")
    return b0.value, w1.value


def soft_table(n_bins: int, unsigned: bool = False):
    """soft_vote over every (dx, dy) in [-255, 255]^2: (b0, w1) uint8[dy+255][dx+255]."""
    b0 = np.empty((511, 511), np.uint8)
    w1 = np.empty((511, 511), np.uint8)
    _check(_load().orc_soft_table(int(n_bins), int(unsigned), _ptr(b0), _ptr(w1)), "soft_table")
    return b0, w1


def soft_bin_map(img: np.ndarray, n_bins: int, unsigned: bool = False):
    """(b0, w1) maps, uint8 h x w each, of an image of shape (h, w) or (h, w, c)."""
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        img = img[:, :, None]
    h, w, c = img.shape
    b0 = np.empty((h, w), np.uint8)
    w1 = np.empty((h, w), np.uint8)
    _check(_load().orc_soft_bin_map(_ptr(img), w, h, c, w * c, n_bins, int(unsigned), _ptr(b0), _ptr(w1)),
           "soft_bin_map")
    return b0, w1


def soft_integral(b0: np.ndarray, w1: np.ndarray, n_bins: int) -> np.ndarray:
    """uint32[n_bins][h+1][w+1]: Eq. 5 over the soft votes (units of 1/SOFT_Q)."""
    b0 = np.ascontiguousarray(b0, np.uint8)
    w1 = np.ascontiguousarray(w1, np.uint8)
    h, w = b0.shape
    out = np.empty((n_bins, h + 1, w + 1), np.uint32)
    _check(_load().orc_soft_integral(_ptr(b0), _ptr(w1), w, h, n_bins, _ptr(out)), "soft_integral")
    return out


def soft_cell_hist(b0: np.ndarray, w1: np.ndarray, n_bins: int, cell: int = 8) -> np.ndarray:
    """uint32[h//cell][w//cell][n_bins]: brute-force vote sums (units of 1/SOFT_Q)."""
    b0 = np.ascontiguousarray(b0, np.uint8)
    w1 = np.ascontiguousarray(w1, np.uint8)
    h, w = b0.shape
    out = np.empty((h // cell, w // cell, n_bins), np.uint32)
    _check(_load().orc_soft_cell_hist(_ptr(b0), _ptr(w1), w, h, n_bins, cell, _ptr(out)),
           "soft_cell_hist")
    return out


def features_from_cells(cells: np.ndarray, p: "ScanParams", wx: int, wy: int) -> np.ndarray:
    """Window feature (Sec. 3.1 / Fig. 4) from a cell-histogram array
    [cy][cx][n] in FP64, in the order of window_feature: raw, the cells in
    row-major order; L2, each 2x2-cell block v / sqrt(|v|^2 + eps^2)."""
    c = cells.astype(np.float64)
    win = c[wy:wy + p.wcy, wx:wx + p.wcx]  # [cy][cx][n]
    if p.norm == 0:
        return win.reshape(-1)
    out = []
    for by in range(p.wcy - 1):
        for bx in range(p.wcx - 1):
            v = np.concatenate([win[by + vv, bx + uu] for vv in (0, 1) for uu in (0, 1)])
            out.append(v / np.sqrt(np.dot(v, v) + p.eps * p.eps))
    return np.concatenate(out)


def soft_score_windows(b0, w1, n_bins, p, tmpl, bias, wxs=None, wys=None):
    """Scores (FP64) of the listed windows under soft votes: features from the
    brute-force vote sums divided by SOFT_Q (a pixel's votes sum to 1).
    Returns (scores [n][K], sum_d |T_d f_d| + |b| [n][K], wxs, wys)."""
    cells = soft_cell_hist(b0, w1, n_bins, p.cell).astype(np.float64) / SOFT_Q
    h, w = b0.shape
    nwx = (w // p.cell) - p.wcx + 1
    nwy = (h // p.cell) - p.wcy + 1
    if wxs is None:
        wys, wxs = np.divmod(np.arange(max(nwx, 0) * max(nwy, 0)), max(nwx, 1))
    T = np.asarray(tmpl, np.float64).reshape(len(bias), -1)
    b = np.asarray(bias, np.float64)
    s = np.empty((len(wxs), len(b)))
    a = np.empty((len(wxs), len(b)))
    for i, (wx, wy) in enumerate(zip(wxs, wys)):
        f = features_from_cells(cells, p, int(wx), int(wy))
        s[i] = T @ f + b
        a[i] = np.abs(T * f[None, :]).sum(axis=1) + np.abs(b)
    return s, a, np.asarray(wxs), np.asarray(wys)


def pyramid(w: int, h: int, scale: float, min_w: int, min_h: int, max_levels: int = 0):
    """[(w_l, h_l, s_l)] of the nearest-neighbour pyramid."""
    cap = 4096
    lw = np.zeros(cap, np.int32)
    lh = np.zeros(cap, np.int32)
    ls = np.zeros(cap, np.float64)
    n = _load().orc_pyramid(w, h, float(scale), min_w, min_h, max_levels, cap,
                            _ptr(lw), _ptr(lh), _ptr(ls))
    _check(n, "pyramid")
    return [(int(lw[i]), int(lh[i]), float(ls[i])) for i in range(n)]


def resize_nn(img: np.ndarray, s: float, lw: int, lh: int) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        img = img[:, :, None]
    h, w, c = img.shape
    out = np.empty((lh, lw, c), dtype=np.uint8)
    _check(_load().orc_resize_nn(_ptr(img), w, h, c, w * c, float(s), lw, lh, _ptr(out)),
           "resize_nn")
    return out


def integral(bins: np.ndarray, n_bins: int) -> np.ndarray:
    """uint32[n_bins][h+1][w+1]; [n][y+1][x+1] = ii_n(x, y)."""
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    h, w = bins.shape
    out = np.empty((n_bins, h + 1, w + 1), dtype=np.uint32)
    _check(_load().orc_integral(_ptr(bins), w, h, n_bins, _ptr(out)), "integral")
    return out


def integral_mod(bins: np.ndarray, n_bins: int, bits: int) -> np.ndarray:
    """Narrow integral images, after the 16-bit integral images the paper
    suggests for small inputs (Sec. 4): [n_bins][h+1][w+1] of uint16 (bits
    16) or uint8 (bits 8) holding the exact Eq. 5 count mod 2^bits. Read as
    modular numbers they serve any image size: the four-corner sum of Eq. 6,
    taken mod 2^bits, still counts a rectangle of fewer than 2^bits pixels
    exactly."""
    if bits not in (16, 8):
        raise ValueError("bits must be 16 or 8")
    full = integral(bins, n_bins)
    return (full & np.uint32((1 << bits) - 1)).astype(np.uint16 if bits == 16 else np.uint8)


def integral_literal(bins: np.ndarray, n_bins: int) -> np.ndarray:
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    h, w = bins.shape
    out = np.empty((n_bins, h + 1, w + 1), dtype=np.uint32)
    _check(_load().orc_integral_literal(_ptr(bins), w, h, n_bins, _ptr(out)),
           "integral_literal")
    return out


def cell_hist(bins: np.ndarray, n_bins: int, cell: int = 8) -> np.ndarray:
    """uint32[h//cell][w//cell][n_bins], brute-force counts."""
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    h, w = bins.shape
    out = np.empty((h // cell, w // cell, n_bins), dtype=np.uint32)
    _check(_load().orc_cell_hist(_ptr(bins), w, h, n_bins, cell, _ptr(out)), "cell_hist")
    return out


class ScanParams:
    """Window geometry: cell size in pixels, window size in cells, block size
    in cells, normalisation (0 raw, 1 L2) and eps."""

    def __init__(self, cell=8, win_cells_x=8, win_cells_y=16, block=2, norm=0, eps=1e-3):
        self.cell, self.wcx, self.wcy = cell, win_cells_x, win_cells_y
        self.block, self.norm, self.eps = block, norm, eps

    def dim(self, n_bins: int) -> int:
        d = _load().orc_feature_dim(n_bins, self.wcx, self.wcy, self.block, self.norm)
        _check(d, "feature_dim")
        return d


def window_grid(w: int, h: int, p: ScanParams):
    a = ctypes.c_int(0)
    b = ctypes.c_int(0)
    _check(_load().orc_window_grid(w, h, p.cell, p.wcx, p.wcy, ctypes.byref(a),
                                   ctypes.byref(b)), "window_grid")
    return a.value, b.value


def window_feature(bins: np.ndarray, n_bins: int, p: ScanParams, wx: int, wy: int):
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    h, w = bins.shape
    out = np.empty(p.dim(n_bins), dtype=np.float64)
    _check(_load().orc_window_feature(_ptr(bins), w, h, n_bins, p.cell, p.wcx, p.wcy, p.block,
                                      p.norm, p.eps, wx, wy, _ptr(out)), "window_feature")
    return out


def score_windows(bins: np.ndarray, n_bins: int, p: ScanParams, tmpl: np.ndarray,
                  bias: np.ndarray, wxs=None, wys=None, want_feats: bool = False):
    """Scores of the listed windows (all windows when wxs/wys are None).

    Returns (scores[n, k], absterms[n, k], feats[n, dim] or None, wxs, wys).
    """
    bins = np.ascontiguousarray(bins, dtype=np.uint8)
    h, w = bins.shape
    tmpl = np.ascontiguousarray(tmpl, dtype=np.float32)
    if tmpl.ndim == 1:
        tmpl = tmpl[None, :]
    bias = np.ascontiguousarray(bias, dtype=np.float32).reshape(-1)
    k = tmpl.shape[0]
    dim = p.dim(n_bins)
    if tmpl.shape[1] != dim or bias.shape[0] != k:
        raise ValueError("template shape does not match the feature length")
    if wxs is None:
        nwx, nwy = window_grid(w, h, p)
        gy, gx = np.meshgrid(np.arange(nwy), np.arange(nwx), indexing="ij")
        wxs, wys = gx.reshape(-1), gy.reshape(-1)
    wxs = np.ascontiguousarray(wxs, dtype=np.int32)
    wys = np.ascontiguousarray(wys, dtype=np.int32)
    n = wxs.shape[0]
    scores = np.empty((n, k), np.float64)
    absterms = np.empty((n, k), np.float64)
    feats = np.empty((n, dim), np.float64) if want_feats else None
    _check(_load().orc_score_windows(_ptr(bins), w, h, n_bins, p.cell, p.wcx, p.wcy, p.block,
                                     p.norm, p.eps, _ptr(tmpl), _ptr(bias), k, n, _ptr(wxs),
                                     _ptr(wys), _ptr(scores),
                                     _ptr(feats) if feats is not None else None,
                                     _ptr(absterms)), "score_windows")
    return scores, absterms, feats, wxs, wys
