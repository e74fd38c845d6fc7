"""The C-ABI library loads, exports every function its header declares, and
rejects bad arguments on the host (no GPU needed: nothing is launched)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2505_05587_amd import _lib as L
from paper_2505_05587_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "steepgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(steepgs_[a-z_0-9]+)\s*\(", src)))


def test_header_symbols_exported():
    names = _declared()
    assert {"steepgs_project", "steepgs_sort", "steepgs_render_fwd", "steepgs_render_bwd_split",
            "steepgs_densify"} <= set(names)
    lib = L.lib()
    for nm in names:
        assert hasattr(lib, nm), nm
    assert L.version().startswith("steepgs")


def test_struct_sizes_match_header():
    assert C.sizeof(L.Camera) == 96
    assert C.sizeof(L.Opts) == 56
    assert C.sizeof(L.SplitSelect) == 40


def test_layout_cameras():
    cams = scenes.make_cameras([(0, 0, 3.0), (1.0, 2.0, 2.0), (0, 3.0, 0.5)], [(979, 546), (64, 64), (17, 9)])
    for tw, th in [(16, 16), (16, 8), (8, 8)]:
        o = L.make_opts(scenes.opts("3dgs", tile_w=tw, tile_h=th))
        arr = (L.Camera * 3)()
        for v in range(3):
            arr[v].width, arr[v].height = int(cams.width[v]), int(cams.height[v])
        tp, tt = L.steepgs_layout_cameras(arr, o)
        tx = (cams.width + tw - 1) // tw
        ty = (cams.height + th - 1) // th
        assert tt == int((tx * ty).sum()) and tp == cams.total_pixels()
        assert [arr[v].tile_offset for v in range(3)] == [0, int(tx[0] * ty[0]), int(tx[0] * ty[0] + tx[1] * ty[1])]
        assert [arr[v].pixel_offset for v in range(3)] == list(cams.pixel_offsets())


def test_bad_arguments_rejected_on_host():
    lib = L.lib()
    o = L.make_opts(scenes.opts("3dgs"))
    # negative sizes, bad SH degree, missing buffers
    assert lib.steepgs_project(None, -1, 0, None, 1, C.byref(o), None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_project(None, 10, 4, None, 1, C.byref(o), None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_project(None, 10, 0, None, 1, C.byref(o), None, None, None, None) == L.ERR_INVALID_ARG
    bad = L.make_opts(scenes.opts("3dgs", tile_w=12))
    assert lib.steepgs_project(None, 10, 0, None, 1, C.byref(bad), None, None, None, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_sort(None, None, None, 10, 1, None, C.byref(o), 0, None, None, 0, None, None, None, None,
                            None, 0, None) == L.ERR_INVALID_ARG
    fake = C.c_void_p(0x1000)
    assert lib.steepgs_render_fwd(fake, 10, fake, fake, fake, 1, C.byref(o), 4, 64, None, fake, fake, fake, None,
                                  None, None, 0, None) == L.ERR_WORKSPACE
    assert lib.steepgs_set_kernel_timer(9, None, None, 0) == L.ERR_INVALID_ARG
    assert lib.steepgs_set_kernel_timer(0, None, None, 0) == L.OK
    assert lib.steepgs_densify(None, 10, 0, None, 1.0, 0.01, 0.0, None, None, 0, None, None, None, None, None, None,
                               0, None) == L.ERR_INVALID_ARG
    sel = L.SplitSelect(None, 1.0, 0.0, 1 << 40, None, 0.0)  # budget beyond 32 bits
    assert lib.steepgs_densify(fake, 10, 0, fake, 1.0, 0.01, 0.0, C.byref(sel), fake, 20, fake, None, None, None,
                               fake, fake, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_adam_step(None, None, None, None, 10, 0, None, None, None, None, None) == L.ERR_INVALID_ARG
    bad = L.make_adam_opts([1e-3] * 6, beta1=1.0)
    assert lib.steepgs_adam_step(fake, fake, fake, fake, 10, 0, C.byref(bad), fake, None, None,
                                 None) == L.ERR_INVALID_ARG
    good = L.make_adam_opts([1e-3] * 6)
    # missing parameter buffers are rejected before anything is enqueued
    assert lib.steepgs_adam_step(None, fake, fake, fake, 10, 0, C.byref(good), fake, None, None,
                                 None) == L.ERR_INVALID_ARG
    assert lib.steepgs_split_remap(fake, 1, 10, fake, fake, 20, None, 0, None) == L.ERR_WORKSPACE
    assert lib.steepgs_split_remap(fake, -1, 10, fake, fake, 20, None, 0, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_render_bwd_split6(fake, 10, 0, fake, 1, C.byref(o), fake, fake, fake, fake, 4, 64, fake, fake,
                                         fake, None, fake, fake, fake, None, fake, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_densify6(None, -1, 0, None, 1.0, 0.01, 0.0, None, 0, None, None, None, None, None, None, 0,
                                None) == L.ERR_INVALID_ARG
    assert lib.steepgs_densify6(fake, 10, 0, fake, 1.0, 0.01, 0.0, fake, 20, fake, None, None, None, fake, None, 0,
                                None) == L.ERR_WORKSPACE
    # the backward's clear on its own, and the backward that skips it
    assert lib.steepgs_render_bwd_clear(-1, 1, fake, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_render_bwd_clear(10, 0, fake, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_render_bwd_clear(10, 1, None, 1 << 20, None) == L.ERR_INVALID_ARG
    assert lib.steepgs_render_bwd_clear(10, 1, fake, 16, None) == L.ERR_WORKSPACE
    assert lib.steepgs_render_bwd_clear(0, 1, fake, 0, None) == L.OK  # nothing to clear
    assert lib.steepgs_render_bwd_split_cleared(fake, 10, 0, fake, 1, C.byref(o), fake, fake, fake, fake, 4, 64, fake,
                                                fake, fake, None, fake, fake, fake, None, fake, 16,
                                                None) == L.ERR_WORKSPACE
    assert lib.steepgs_render_bwd_split_cleared(fake, 10, 4, fake, 1, C.byref(o), fake, fake, fake, fake, 4, 64, fake,
                                                fake, fake, None, fake, fake, fake, None, fake, 1 << 30,
                                                None) == L.ERR_INVALID_ARG
    assert lib.steepgs_status_string(2) == b"output capacity exceeded"


def test_workspace_sizes_grow_with_problem():
    a = L.steepgs_workspace_size(L.STAGE_SORT, 1000, 1, 10000)
    b = L.steepgs_workspace_size(L.STAGE_SORT, 1000, 2, 20000)
    assert 0 < a < b
    assert L.steepgs_workspace_size(L.STAGE_RENDER_BWD, 1000, 4) >= 9 * 4 * 1000 * 4
    assert L.steepgs_workspace_size(L.STAGE_DENSIFY, 1000, 1) >= 1000 * 4 * 6
