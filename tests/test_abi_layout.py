"""The binding's ctypes structures have the C header's layout: a C program
compiled against include/hog.h prints every struct's size and each field's
offset and size under the names the binding uses; they must equal what
ctypes computes. A field renamed, added or reordered on one side only fails
to compile or differs here."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1703_06256_amd import hog

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [
    ("hog_scan_params", hog.ScanParams),
    ("hog_plan_desc", hog.PlanDesc),
    ("hog_level_info", hog.LevelInfo),
    ("hog_image_info", hog.ImageInfo),
    ("hog_plan_sizes", hog.PlanSizes),
    ("hog_tiles", hog.Tiles),
    ("hog_server_config", hog.ServerConfig),
]


def _c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hog.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'    printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname}.{f} %zu %zu\\n", offsetof({cname}, {f}), '
                         f'sizeof((({cname} *)0)->{f}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return dict((k, v) for k, v in (ln.split(" ", 1) for ln in out.splitlines()))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_the_header(tmp_path):
    c = _c_layout(tmp_path)
    for cname, cls in PAIRS:
        assert int(c[cname]) == ctypes.sizeof(cls), cname
        for f, t in cls._fields_:
            off, size = map(int, c[f"{cname}.{f}"].split())
            assert off == getattr(cls, f).offset, f"{cname}.{f} offset"
            assert size == ctypes.sizeof(t), f"{cname}.{f} size"


CONSTANTS = {  # header name -> binding name
    **{n: n for n in ("HOG_OK", "HOG_E_INVALID", "HOG_E_NOMEM", "HOG_E_DEVICE", "HOG_E_BUSY",
                      "HOG_E_NOT_READY", "HOG_NO_BIN", "HOG_NORM_RAW", "HOG_NORM_L2",
                      "HOG_ORIENT_SIGNED", "HOG_ORIENT_UNSIGNED", "HOG_VOTES_HARD", "HOG_VOTES_SOFT",
                      "HOG_SOFT_QUANTUM", "HOG_MAX_LEVEL_GROUPS", "HOG_LUT_DEVICE_FULL",
                      "HOG_LUT_DEVICE_HALF", "HOG_LUT_DEVICE_SOFT", "HOG_STATIC_SCRATCH_BYTES")},
    "HOG_LUT_SIDE": "LUT_SIDE",
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_header_constants_match_the_binding(tmp_path):
    """Every enum value and #define the binding mirrors, as the C compiler
    sees it through the header."""
    lines = ['#include <stdio.h>', '#include "hog.h"', "int main(void) {"]
    lines += [f'    printf("{c} %d\\n", (int)({c}));' for c in CONSTANTS]
    lines += ["    return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "consts"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict((k, int(v)) for k, v in (ln.split() for ln in out.splitlines()))
    for c, py in CONSTANTS.items():
        assert got[c] == getattr(hog, py), c
