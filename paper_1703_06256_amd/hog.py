"""Python binding of libhog (include/hog.h): argument marshalling only.

Every function here forwards to the C ABI function of the same name; all
arithmetic happens in the library's HIP kernels. PyTorch supplies device
memory (tensors, passed by data_ptr) and streams (the current stream unless
one is given). If libhog.so has not been built, the first call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhog.so")

HOG_OK, HOG_E_INVALID, HOG_E_NOMEM, HOG_E_DEVICE, HOG_E_BUSY, HOG_E_NOT_READY = range(6)
HOG_NO_BIN = 255
HOG_NORM_RAW, HOG_NORM_L2 = 0, 1
HOG_ORIENT_SIGNED, HOG_ORIENT_UNSIGNED = 0, 1
HOG_VOTES_HARD, HOG_VOTES_SOFT = 0, 1
HOG_SOFT_QUANTUM = 32
HOG_MAX_LEVEL_GROUPS = 4
HOG_LUT_DEVICE_FULL, HOG_LUT_DEVICE_HALF, HOG_LUT_DEVICE_SOFT = 0, 1, 2
HOG_STATIC_SCRATCH_BYTES = 64 << 20
LUT_SIDE = 511

# Every symbol include/hog.h declares.
EXPORTS = (
    "hog_last_error", "hog_lut_fill_host", "hog_lut_build", "hog_lut_free", "hog_lut_bins",
    "hog_lut_host", "hog_lut_read_device", "hog_lut_fill_host_ex", "hog_lut_build_ex", "hog_lut_orientation",
    "hog_lut_fill_soft_host", "hog_plan_create", "hog_plan_create_batch", "hog_plan_images",
    "hog_plan_get_image", "hog_plan_destroy", "hog_plan_get_sizes",
    "hog_plan_get_level", "hog_bin_map", "hog_integral", "hog_scan_windows", "hog_run", "hog_run_static",
    "hog_graph_create", "hog_graph_launch", "hog_graph_destroy", "hog_plan_get_tiles",
    "hog_plan_set_tiles", "hog_plan_autotune", "hog_tune_cache_open", "hog_tune_cache_stats",
    "hog_server_create", "hog_server_destroy",
    "hog_server_warm", "hog_submit", "hog_poll", "hog_wait_any",
    "hog_timing_enable", "hog_timing_reset", "hog_timing_get",
)


class HogError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libhog status {status}: {msg}")
        self.status = status


class ScanParams(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("win_cells_x", ctypes.c_int32),
                ("win_cells_y", ctypes.c_int32), ("block", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("eps", ctypes.c_float)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("scale", ctypes.c_double),
                ("n_templates", ctypes.c_int32), ("scan", ScanParams),
                ("plane_bits", ctypes.c_int32), ("votes", ctypes.c_int32)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("scale", ctypes.c_double), ("bins_offset", ctypes.c_int64),
                ("bins_pitch", ctypes.c_int64), ("ii_offset", ctypes.c_int64),
                ("ii_pitch", ctypes.c_int64), ("ii_plane_stride", ctypes.c_int64),
                ("cells_x", ctypes.c_int32), ("cells_y", ctypes.c_int32),
                ("windows_x", ctypes.c_int32), ("windows_y", ctypes.c_int32),
                ("score_offset", ctypes.c_int64), ("cell_offset", ctypes.c_int64),
                ("block_offset", ctypes.c_int64)]


class ImageInfo(ctypes.Structure):
    _fields_ = [("first_level", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("img_offset", ctypes.c_int64), ("img_pitch", ctypes.c_int64),
                ("total_pixels", ctypes.c_int64), ("total_windows", ctypes.c_int64)]


class Tiles(ctypes.Structure):
    _fields_ = [("bin_chunk", ctypes.c_int32), ("score_rows", ctypes.c_int32),
                ("level_groups", ctypes.c_int32), ("lut_global", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("n_templates", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("scale", ctypes.c_double), ("scan", ScanParams),
                ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32),
                ("memory_budget", ctypes.c_int64), ("host_budget", ctypes.c_int64),
                ("max_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("orientation", ctypes.c_int32),
                ("votes", ctypes.c_int32), ("plane_bits", ctypes.c_int32),
                ("copy_threads", ctypes.c_int32)]


class PlanSizes(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("bins_bytes", ctypes.c_int64),
                ("ii_elems", ctypes.c_int64), ("score_elems", ctypes.c_int64),
                ("cell_elems", ctypes.c_int64), ("block_elems", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("feature_dim", ctypes.c_int32),
                ("total_pixels", ctypes.c_int64), ("total_windows", ctypes.c_int64),
                ("ii_elem_bytes", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libhog.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1703_06256_amd.build` (there is no fallback path)")
    # One HIP runtime per process. PyTorch ships its own copy of the HIP
    # runtime under the same soname as the system's; with torch loaded first
    # the dynamic linker binds libhog to that copy, so torch's device memory
    # and stream handles belong to the runtime libhog calls. Loaded the other
    # way round, the process would hold two runtimes and torch's would find
    # no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    sig = {
        "hog_last_error": ([], ctypes.c_char_p),
        "hog_lut_fill_host": ([i32, vp], i32),
        "hog_lut_build": ([i32, ctypes.POINTER(vp)], i32),
        "hog_lut_fill_host_ex": ([i32, i32, vp], i32),
        "hog_lut_build_ex": ([i32, i32, ctypes.POINTER(vp)], i32),
        "hog_lut_orientation": ([vp], i32),
        "hog_lut_fill_soft_host": ([i32, i32, vp], i32),
        "hog_lut_free": ([vp], None),
        "hog_lut_bins": ([vp], i32),
        "hog_lut_host": ([vp], vp),
        "hog_lut_read_device": ([vp, i32, vp, i64], i32),
        "hog_plan_create": ([ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)], i32),
        "hog_plan_create_batch": ([ctypes.POINTER(PlanDesc), i32, ctypes.POINTER(vp)], i32),
        "hog_plan_images": ([vp], i32),
        "hog_plan_get_image": ([vp, i32, ctypes.POINTER(ImageInfo)], i32),
        "hog_plan_destroy": ([vp], None),
        "hog_plan_get_sizes": ([vp, ctypes.POINTER(PlanSizes)], i32),
        "hog_plan_get_level": ([vp, i32, ctypes.POINTER(LevelInfo)], i32),
        "hog_bin_map": ([vp, vp, vp, i64, vp, vp], i32),
        "hog_integral": ([vp, vp, vp, vp, vp], i32),
        "hog_scan_windows": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "hog_run": ([vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp], i32),
        "hog_run_static": ([vp, vp, vp, i64, vp, vp, vp, vp, vp, vp], i32),
        "hog_graph_create": ([vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)], i32),
        "hog_graph_launch": ([vp, vp], i32),
        "hog_graph_destroy": ([vp], None),
        "hog_plan_get_tiles": ([vp, ctypes.POINTER(Tiles)], i32),
        "hog_server_create": ([ctypes.POINTER(ServerConfig), vp, vp, ctypes.POINTER(vp)], i32),
        "hog_server_destroy": ([vp], None),
        "hog_submit": ([vp, vp, i32, i32, ctypes.POINTER(ctypes.c_uint64)], i32),
        "hog_poll": ([vp, ctypes.c_uint64, vp, ctypes.c_size_t, ctypes.POINTER(i32),
                      ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], i32),
        "hog_server_warm": ([vp, i32, i32], i32),
        "hog_wait_any": ([vp, ctypes.POINTER(ctypes.c_uint64), i32, i64, ctypes.POINTER(i32)], i32),
        "hog_plan_set_tiles": ([vp, ctypes.POINTER(Tiles)], i32),
        "hog_plan_autotune": ([vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, i32,
                               ctypes.POINTER(Tiles)], i32),
        "hog_tune_cache_open": ([ctypes.c_char_p], i32),
        "hog_tune_cache_stats": ([ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "hog_timing_enable": ([i32], i32),
        "hog_timing_reset": ([], i32),
        "hog_timing_get": ([ctypes.c_char_p, ctypes.POINTER(i64),
                            ctypes.POINTER(ctypes.c_double)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != HOG_OK:
        raise HogError(status, load_library().hog_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, min_elems: int, name: str):
    """Device pointer of a contiguous CUDA tensor of the given dtype and size."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < min_elems:
        raise ValueError(f"{name} has {t.numel()} elements, needs {min_elems}")
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------------------------
def hog_lut_fill_host(n_bins: int, orientation: int = HOG_ORIENT_SIGNED) -> np.ndarray:
    """Host-only table: uint8[dy+255][dx+255]."""
    out = np.empty((LUT_SIDE, LUT_SIDE), np.uint8)
    _check(load_library().hog_lut_fill_host_ex(int(n_bins), int(orientation),
                                               out.ctypes.data_as(ctypes.c_void_p)))
    return out


def hog_lut_fill_soft_host(n_bins: int, orientation: int = HOG_ORIENT_SIGNED):
    """Host-only soft-vote table: (b0, w1) as two uint8[dy+255][dx+255]."""
    out = np.empty((LUT_SIDE, LUT_SIDE), np.uint16)
    _check(load_library().hog_lut_fill_soft_host(int(n_bins), int(orientation),
                                                 out.ctypes.data_as(ctypes.c_void_p)))
    return (out & 255).astype(np.uint8), (out >> 8).astype(np.uint8)


class Lut:
    """Library-owned lookup table (host + device copies)."""

    def __init__(self, handle, n_bins):
        self.handle = handle
        self.n_bins = n_bins

    def host_table(self) -> np.ndarray:
        p = load_library().hog_lut_host(self.handle)
        buf = (ctypes.c_uint8 * (LUT_SIDE * LUT_SIDE)).from_address(p)
        return np.frombuffer(buf, dtype=np.uint8).reshape(LUT_SIDE, LUT_SIDE).copy()

    def device_table(self, table: int) -> np.ndarray:
        """A device copy read back: HOG_LUT_DEVICE_FULL uint8[511][511],
        HOG_LUT_DEVICE_HALF uint8[256][511], HOG_LUT_DEVICE_SOFT uint16[511][511]."""
        shape, dt = {HOG_LUT_DEVICE_FULL: ((LUT_SIDE, LUT_SIDE), np.uint8),
                     HOG_LUT_DEVICE_HALF: ((256, LUT_SIDE), np.uint8),
                     HOG_LUT_DEVICE_SOFT: ((LUT_SIDE, LUT_SIDE), np.uint16)}[table]
        out = np.empty(shape, dt)
        _check(load_library().hog_lut_read_device(self.handle, int(table), out.ctypes.data_as(ctypes.c_void_p),
                                                  out.nbytes))
        return out

    def free(self):
        if self.handle:
            load_library().hog_lut_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def hog_lut_build(n_bins: int, orientation: int = HOG_ORIENT_SIGNED) -> Lut:
    h = ctypes.c_void_p()
    _check(load_library().hog_lut_build_ex(int(n_bins), int(orientation), ctypes.byref(h)))
    return Lut(h, int(n_bins))


def make_desc(width, height, channels=1, n_bins=8, max_levels=1, scale=1.0, n_templates=1,
              cell=8, win_cells_x=8, win_cells_y=16, block=2, norm=HOG_NORM_RAW,
              eps=1e-3, plane_bits=32, votes=HOG_VOTES_HARD) -> PlanDesc:
    return PlanDesc(width, height, channels, n_bins, max_levels, scale, n_templates,
                    ScanParams(cell, win_cells_x, win_cells_y, block, norm, eps), plane_bits, votes)


def ii_dtype(plan: "Plan"):
    """torch dtype holding the plan's plane elements (same bits: int32 for
    uint32, int16 for uint16, uint8)."""
    import torch
    return {4: torch.int32, 2: torch.int16, 1: torch.uint8}[plan.sizes.ii_elem_bytes]


class Plan:
    """Level geometry and buffer layout for one image shape, or (batch) for a
    list of images packed in one input buffer."""

    def __init__(self, desc, batch: bool = False):
        h = ctypes.c_void_p()
        if batch:
            descs = list(desc)
            arr = (PlanDesc * len(descs))(*descs)
            _check(load_library().hog_plan_create_batch(arr, len(descs), ctypes.byref(h)))
            self.desc = descs[0]
            self.descs = descs
        else:
            _check(load_library().hog_plan_create(ctypes.byref(desc), ctypes.byref(h)))
            self.desc = desc
            self.descs = [desc]
        self.batch = batch
        self.handle = h
        self.images = []
        for i in range(load_library().hog_plan_images(h)):
            ii = ImageInfo()
            _check(load_library().hog_plan_get_image(h, i, ctypes.byref(ii)))
            self.images.append(ii)
        sz = PlanSizes()
        _check(load_library().hog_plan_get_sizes(h, ctypes.byref(sz)))
        self.sizes = sz
        self.levels = []
        for l in range(sz.n_levels):
            li = LevelInfo()
            _check(load_library().hog_plan_get_level(h, l, ctypes.byref(li)))
            self.levels.append(li)

    def destroy(self):
        if self.handle:
            load_library().hog_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hog_bin_map(plan: Plan, lut: Lut, img, bins, stream=None, img_pitch=None):
    import torch
    d = plan.desc
    if plan.batch:
        pitch = 0
        last = plan.images[-1]
        need = last.img_offset + last.height * last.img_pitch
    else:
        pitch = d.width * d.channels if img_pitch is None else int(img_pitch)
        need = (d.height - 1) * pitch + d.width * d.channels
    _check(load_library().hog_bin_map(
        plan.handle, lut.handle, _dptr(img, torch.uint8, need, "img"), pitch,
        _dptr(bins, torch.uint8, plan.sizes.bins_bytes, "bins"), _stream(stream)))


def hog_integral(plan: Plan, bins, ii, workspace, stream=None):
    import torch
    _check(load_library().hog_integral(
        plan.handle, _dptr(bins, torch.uint8, plan.sizes.bins_bytes, "bins"),
        _dptr(ii, ii_dtype(plan), plan.sizes.ii_elems, "ii"),
        _dptr(workspace, torch.uint8, plan.sizes.workspace_bytes, "workspace"),
        _stream(stream)))


def hog_scan_windows(plan: Plan, ii, tmpl, bias, scores, workspace, cell_hist=None,
                     block_feat=None, stream=None):
    import torch
    k = plan.desc.n_templates
    _check(load_library().hog_scan_windows(
        plan.handle, _dptr(ii, ii_dtype(plan), plan.sizes.ii_elems, "ii") if ii is not None else None,
        _dptr(tmpl, torch.float32, k * plan.sizes.feature_dim, "tmpl"),
        _dptr(bias, torch.float32, k, "bias"),
        _dptr(scores, torch.float32, plan.sizes.score_elems, "scores"),
        _dptr(cell_hist, torch.int32, plan.sizes.cell_elems, "cell_hist"),
        _dptr(block_feat, torch.float32, plan.sizes.block_elems, "block_feat"),
        _dptr(workspace, torch.uint8, plan.sizes.workspace_bytes, "workspace"),
        _stream(stream)))


def hog_timing_enable(on: bool):
    _check(load_library().hog_timing_enable(1 if on else 0))


def hog_timing_reset():
    _check(load_library().hog_timing_reset())


def hog_timing_get(kernel: str):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load_library().hog_timing_get(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def pack_images(plan: Plan, images) -> np.ndarray:
    """Host buffer holding a batch plan's images (uint8 HWC arrays) packed as
    hog_bin_map reads them."""
    assert plan.batch and len(images) == len(plan.images)
    last = plan.images[-1]
    out = np.zeros(last.img_offset + last.height * last.img_pitch, np.uint8)
    for im, info in zip(images, plan.images):
        a = np.ascontiguousarray(im).reshape(-1)
        assert a.size == info.height * info.img_pitch
        out[info.img_offset: info.img_offset + a.size] = a
    return out


class Buffers:
    """Device buffers (torch tensors) sized for a plan. uint32 data is held in
    int32 tensors (same bits); use .view or & 0xffffffff to read counts."""

    def __init__(self, plan: Plan, device="cuda", cell_hist=False, block_feat=False):
        import torch
        s = plan.sizes
        self.bins = torch.empty(max(s.bins_bytes, 1), dtype=torch.uint8, device=device)
        self.ii = torch.empty(max(s.ii_elems, 1), dtype=ii_dtype(plan), device=device)
        self.scores = torch.empty(max(s.score_elems, 1), dtype=torch.float32, device=device)
        self.workspace = torch.empty(max(s.workspace_bytes, 1), dtype=torch.uint8, device=device)
        self.cell_hist = (torch.empty(max(s.cell_elems, 1), dtype=torch.int32, device=device)
                          if cell_hist else None)
        self.block_feat = (torch.empty(max(s.block_elems, 1), dtype=torch.float32, device=device)
                           if block_feat else None)


def run_path(plan: Plan, lut: Lut, img, tmpl, bias, buf: Buffers, stream=None,
             cells_from_planes: bool = False):
    """The whole hot path: hog_bin_map, hog_integral, hog_scan_windows. By
    default the scorer uses the cell histograms hog_integral cached (8-pixel
    cells); with cells_from_planes, or other cell sizes, it recomputes them
    from the integral images."""
    hog_bin_map(plan, lut, img, buf.bins, stream)
    hog_integral(plan, buf.bins, buf.ii, buf.workspace, stream)
    from_planes = cells_from_planes or plan.desc.scan.cell != 8
    hog_scan_windows(plan, buf.ii if from_planes else None, tmpl, bias, buf.scores,
                     buf.workspace, buf.cell_hist, buf.block_feat, stream)


def _run_args(plan: Plan, lut: Lut, img, tmpl, bias, buf: "Buffers", img_pitch=None, with_workspace=True):
    import torch
    d = plan.desc
    if plan.batch:
        pitch = 0
        last = plan.images[-1]
        need = last.img_offset + last.height * last.img_pitch
    else:
        pitch = d.width * d.channels if img_pitch is None else int(img_pitch)
        need = (d.height - 1) * pitch + d.width * d.channels
    k = d.n_templates
    args = (plan.handle, lut.handle, _dptr(img, torch.uint8, need, "img"), pitch,
            _dptr(buf.bins, torch.uint8, plan.sizes.bins_bytes, "bins"),
            _dptr(buf.ii, ii_dtype(plan), plan.sizes.ii_elems, "ii"),
            _dptr(tmpl, torch.float32, k * plan.sizes.feature_dim, "tmpl"),
            _dptr(bias, torch.float32, k, "bias"),
            _dptr(buf.scores, torch.float32, plan.sizes.score_elems, "scores"))
    if with_workspace:
        args += (_dptr(buf.workspace, torch.uint8, plan.sizes.workspace_bytes, "workspace"),)
    return args


def hog_run(plan: Plan, lut: Lut, img, tmpl, bias, buf: "Buffers", stream=None, img_pitch=None):
    """The whole path in one C call (hog_run)."""
    _check(load_library().hog_run(*_run_args(plan, lut, img, tmpl, bias, buf, img_pitch), _stream(stream)))


def hog_run_static(plan: Plan, lut: Lut, img, tmpl, bias, buf: "Buffers", stream=None, img_pitch=None):
    """hog_run on the library's static scratch (no workspace; buf.workspace is
    not used and may be None)."""
    args = _run_args(plan, lut, img, tmpl, bias, buf, img_pitch, with_workspace=False)
    _check(load_library().hog_run_static(*args, _stream(stream)))


def plan_tiles(plan: Plan) -> Tiles:
    t = Tiles()
    _check(load_library().hog_plan_get_tiles(plan.handle, ctypes.byref(t)))
    return t


def set_plan_tiles(plan: Plan, bin_chunk: int, score_rows: int = 0, level_groups: int = 1,
                   lut_global: int = 0):
    t = Tiles(bin_chunk, score_rows, level_groups, lut_global)
    _check(load_library().hog_plan_set_tiles(plan.handle, ctypes.byref(t)))


def autotune(plan: Plan, lut: Lut, img, tmpl, bias, buf: "Buffers", stream=None, reps=3,
             img_pitch=None) -> Tiles:
    t = Tiles()
    _check(load_library().hog_plan_autotune(*_run_args(plan, lut, img, tmpl, bias, buf, img_pitch),
                                            _stream(stream), int(reps), ctypes.byref(t)))
    return t


def tune_cache_open(path) -> None:
    """hog_tune_cache_open: keep autotune results in the text file at path
    (None closes the cache)."""
    _check(load_library().hog_tune_cache_open(None if path is None else os.fsencode(path)))


def tune_cache_stats():
    """(hits, misses, entries) of the autotune cache since it was opened."""
    h, m, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().hog_tune_cache_stats(ctypes.byref(h), ctypes.byref(m), ctypes.byref(e)))
    return h.value, m.value, e.value


class Server:
    """hog_server_*: a request queue with continuous batching on the current
    device. tmpl float32 [K][D] and bias float32 [K] are host arrays."""

    def __init__(self, tmpl: np.ndarray, bias: np.ndarray, channels=3, n_bins=8, max_levels=1,
                 scale=1.0, cell=8, win_cells_x=8, win_cells_y=16, block=2, norm=HOG_NORM_L2,
                 eps=1e-3, max_width=1920, max_height=1080, memory_budget=1 << 30, host_budget=None,
                 max_slots=16, max_batch=8, max_queue=1024, streams=3, copy_threads=4,
                 orientation=HOG_ORIENT_SIGNED, votes=HOG_VOTES_HARD, plane_bits=32):
        if host_budget is None:
            host_budget = 4 * max_batch * max_width * max_height * channels
        self._tmpl = np.ascontiguousarray(tmpl, np.float32)
        self._bias = np.ascontiguousarray(bias, np.float32)
        self.k = self._bias.size
        self.channels = channels
        self.max_levels = max_levels
        cfg = ServerConfig(channels, n_bins, self.k, max_levels, scale,
                           ScanParams(cell, win_cells_x, win_cells_y, block, norm, eps),
                           max_width, max_height, memory_budget, host_budget, max_slots, max_batch,
                           max_queue, streams, orientation, votes, plane_bits, copy_threads)
        h = ctypes.c_void_p()
        _check(load_library().hog_server_create(
            ctypes.byref(cfg), self._tmpl.ctypes.data_as(ctypes.c_void_p),
            self._bias.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.handle = h

    def warm(self, w: int, h: int):
        """Build the batch plans for 1..max_batch images of w x h now."""
        _check(load_library().hog_server_warm(self.handle, w, h))

    def submit(self, img: np.ndarray) -> int:
        a = np.ascontiguousarray(img, np.uint8)
        h, w = a.shape[0], a.shape[1]
        t = ctypes.c_uint64()
        _check(load_library().hog_submit(self.handle, a.ctypes.data_as(ctypes.c_void_p), w, h,
                                         ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, cap: int, out: np.ndarray = None):
        """None while not ready; else (scores, nwx, nwy, latency_s): scores is
        float32[nwy * nwx * K] for single-level servers, else the cap floats
        written (every level, in order). `out` (float32, >= cap) avoids an
        allocation per call."""
        if out is None:
            out = np.empty(max(cap, 1), np.float32)
        nwx, nwy, lat = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        st = load_library().hog_poll(self.handle, ctypes.c_uint64(ticket),
                                     out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(nwx),
                                     ctypes.byref(nwy), ctypes.byref(lat))
        if st == HOG_E_NOT_READY:
            return None
        _check(st)
        if self.max_levels == 1:
            out = out[:nwx.value * nwy.value * self.k]
        return out, nwx.value, nwy.value, lat.value

    def wait_any(self, timeout_us: int = 0, cap: int = 256) -> list:
        """Tickets finished since the last call (hog_wait_any), waiting up to
        timeout_us while there are none."""
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int()
        _check(load_library().hog_wait_any(self.handle, buf, cap, int(timeout_us), ctypes.byref(n)))
        return list(buf[:n.value])

    def close(self):
        if self.handle:
            load_library().hog_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """hog_run captured into a HIP graph for fixed buffers (hog_graph_*)."""

    def __init__(self, plan: Plan, lut: Lut, img, tmpl, bias, buf: "Buffers", img_pitch=None):
        h = ctypes.c_void_p()
        _check(load_library().hog_graph_create(*_run_args(plan, lut, img, tmpl, bias, buf, img_pitch),
                                               ctypes.byref(h)))
        self.handle = h
        self._keep = (plan, lut, img, tmpl, bias, buf)  # buffers must outlive the graph

    def launch(self, stream=None):
        _check(load_library().hog_graph_launch(self.handle, _stream(stream)))

    def destroy(self):
        if self.handle:
            load_library().hog_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# Views of one level inside the plan-layout buffers (host numpy arrays).
def level_bins(plan: Plan, bins_host: np.ndarray, l: int):
    """uint8[h][w] bins of level l; soft votes: the pair (b0, w1) of uint8[h][w]."""
    li = plan.levels[l]
    a = bins_host[li.bins_offset: li.bins_offset + li.bins_pitch * li.height]
    a = a.reshape(li.height, li.bins_pitch)
    if plan.desc.votes == HOG_VOTES_SOFT:
        e = a[:, :2 * li.width].reshape(li.height, li.width, 2)
        return e[:, :, 0].copy(), e[:, :, 1].copy()
    return a[:, :li.width]


def level_planes(plan: Plan, ii_host: np.ndarray, l: int) -> np.ndarray:
    """uint32 / uint16 / uint8 [n_bins][h][w] of level l: [n][y][x] = ii_n(x, y)
    (mod 2^plane_bits)."""
    li = plan.levels[l]
    nb = plan.desc.n_bins
    et = {4: np.uint32, 2: np.uint16, 1: np.uint8}[plan.sizes.ii_elem_bytes]
    a = ii_host.view(et)[li.ii_offset: li.ii_offset + li.ii_plane_stride * nb]
    a = a.reshape(nb, li.ii_plane_stride)[:, :li.ii_pitch * li.height]
    return a.reshape(nb, li.height, li.ii_pitch)[:, :, :li.width]


def level_scores(plan: Plan, scores_host: np.ndarray, l: int) -> np.ndarray:
    """float32[windows_y][windows_x][K] of level l."""
    li = plan.levels[l]
    k = plan.desc.n_templates
    n = li.windows_x * li.windows_y * k
    return scores_host[li.score_offset: li.score_offset + n].reshape(li.windows_y, li.windows_x, k)


def level_cells(plan: Plan, cell_host: np.ndarray, l: int) -> np.ndarray:
    li = plan.levels[l]
    nb = plan.desc.n_bins
    n = li.cells_x * li.cells_y * nb
    return cell_host.view(np.uint32)[li.cell_offset: li.cell_offset + n].reshape(
        li.cells_y, li.cells_x, nb)


def level_blocks(plan: Plan, block_host: np.ndarray, l: int) -> np.ndarray:
    """float32[cells_y-1][cells_x-1][4][n_bins] of level l (L2 plans)."""
    li = plan.levels[l]
    nb = plan.desc.n_bins
    bw, bh = li.cells_x - 1, li.cells_y - 1
    if bw < 1 or bh < 1:
        return np.zeros((0, 0, 4, nb), np.float32)
    n = bw * bh * 4 * nb
    return block_host[li.block_offset: li.block_offset + n].reshape(bh, bw, 4, nb)
