"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before touching the GPU.  CPU only (no kernel is launched)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_10148_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sss():
    from paper_2503_10148_amd import build, sss as binding
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sss.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sss_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for fn in ("sss_project", "sss_bin_sort", "sss_render_fwd", "sss_render_bwd", "sss_sghmc_step"):
        assert fn in names


def test_library_exports_every_declared_symbol(sss):
    lib = ctypes.CDLL(sss.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sss.lib().sss_version() == 106


def test_default_options(sss):
    o = sss.render_opts()
    assert o.alpha_min == pytest.approx(1 / 255)
    assert o.alpha_max == pytest.approx(0.99)
    assert o.t_min == pytest.approx(1e-4)
    assert (o.nu_min, o.nu_max, o.lowpass) == (1.0, 1e4, 0.0)


def test_tiles_and_pixels_of_ragged_views(sss):
    cams = [scenes.ring_camera(1297, 840), scenes.ring_camera(17, 16), scenes.ring_camera(1, 1)]
    assert sss.total_tiles(cams) == 82 * 53 + 2 * 1 + 1
    assert sss.total_pixels(cams) == 1297 * 840 + 17 * 16 + 1


def test_workspace_sizes_grow(sss):
    L = sss.lib()
    a = L.sss_bin_sort_workspace(1000, 1000)
    b = L.sss_bin_sort_workspace(1000, 10 ** 6)
    assert 0 < a < b
    assert L.sss_render_bwd_workspace(1000, 0) == 1000 * 12 * 8 + 16  # FP64 per-entry sums, work counter
    assert L.sss_render_bwd_workspace(1000, 100) >= 1000 * 12 * 8 + 800    # + loss and order per tile


def _scene_struct(sss, n=10, deg=0, null=None):
    ptrs = [ctypes.c_void_p(0x1000 + 64 * i) for i in range(6)]
    if null is not None:
        ptrs[null] = ctypes.c_void_p(0)
    return sss.Scene(n, deg, 0, *ptrs)


def _proj_struct(sss):
    return sss.Proj(0x2000, 0x3000, 0x5000)


@pytest.mark.parametrize("kind", ["null_scene", "bad_degree", "zero_n", "null_array", "no_views", "too_many_views",
                                  "zero_width", "bad_focal", "bad_opts", "alpha_max_one"])
def test_project_rejects_bad_arguments(sss, kind):
    L = sss.lib()
    cam = scenes.ring_camera(64, 48)
    cams = sss.camera_array([cam] * 17)
    opts = sss.render_opts()
    scene = _scene_struct(sss)
    nviews = 1
    if kind == "bad_degree":
        scene = _scene_struct(sss, deg=4)
    elif kind == "zero_n":
        scene = _scene_struct(sss, n=0)
    elif kind == "null_array":
        scene = _scene_struct(sss, null=5)
    elif kind == "no_views":
        nviews = 0
    elif kind == "too_many_views":
        nviews = 17
    elif kind == "zero_width":
        cams[0].width = 0
    elif kind == "bad_focal":
        cams[0].fx = 0.0
    elif kind == "bad_opts":
        opts.nu_min = 0.5
    elif kind == "alpha_max_one":
        opts.alpha_max = 1.0      # 1 - alpha must stay positive
    p = _proj_struct(sss)
    sp = None if kind == "null_scene" else ctypes.byref(scene)
    rc = L.sss_project(sp, cams, nviews, ctypes.byref(opts), ctypes.byref(p), None)
    assert rc == sss.ERR_INVALID
    assert len(L.sss_last_error()) > 0


def test_bin_sort_rejects_short_workspace_and_nulls(sss):
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    p = _proj_struct(sss)
    b = sss.Bins(0x1000, 0x2000, 0x3000, 0x4000, None, None, None, 100, 0, 0)
    assert L.sss_bin_sort(ctypes.byref(p), cams, 1, 10, ctypes.byref(b), None, 0, None) == sss.ERR_INVALID
    b0 = sss.Bins(0, 0x2000, 0x3000, 0x4000, None, None, None, 100, 0, 0)
    assert L.sss_bin_sort(ctypes.byref(p), cams, 1, 10, ctypes.byref(b0), ctypes.c_void_p(0x9000), 10 ** 9,
                          None) == sss.ERR_INVALID


def test_render_bwd_rejects_unknown_mode_and_short_workspace(sss):
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    opts = sss.render_opts()
    scene = _scene_struct(sss)
    p = _proj_struct(sss)
    b = sss.Bins(0x1000, 0x2000, 0x3000, 0x4000, None, None, None, 100, 0, 0)
    g = sss.Grads(0, 0, 0, 0, 0, 0, 0, 0)
    args = lambda mode, loss, wsb: (ctypes.byref(scene), ctypes.byref(p), ctypes.byref(b), cams, 1,
                                    ctypes.byref(opts), mode, loss, ctypes.c_void_p(0x6000), ctypes.c_void_p(0x7000),
                                    ctypes.c_void_p(0x8000), None, None, ctypes.byref(g), ctypes.c_void_p(0x9000),
                                    wsb, None)
    assert L.sss_render_bwd(*args(7, 0, 10 ** 6)) == sss.ERR_INVALID
    assert L.sss_render_bwd(*args(0, 9, 10 ** 6)) == sss.ERR_INVALID
    assert L.sss_render_bwd(*args(0, 0, 10)) == sss.ERR_INVALID
    assert b"workspace" in L.sss_last_error()
    assert L.sss_render_bwd(*args(8, 0, 10 ** 6)) == sss.ERR_INVALID          # unknown flag bit
    # deterministic mode without the rank offsets of the bin sort
    assert L.sss_render_bwd(*args(sss.BWD_DETERMINISTIC, 0, 10 ** 9)) == sss.ERR_INVALID
    assert b"rank_offset" in L.sss_last_error()
    b.rank_offset = 0x5000
    b.n_pairs, b.n_visible = 100, 10
    assert L.sss_render_bwd(*args(sss.BWD_DETERMINISTIC | sss.BWD_RECOMPUTE, 0, 100)) == sss.ERR_INVALID
    assert b"workspace" in L.sss_last_error()


def test_deterministic_workspace_covers_pairs_and_tiles(sss):
    L = sss.lib()
    base = L.sss_render_bwd_workspace_det(1000, 0, 10)
    assert base >= 1000 * 48
    assert L.sss_render_bwd_workspace_det(1000, 10 ** 6, 10) - base >= 10 ** 6 * 48 - 48 - 256
    assert L.sss_render_bwd_workspace_det(1000, 0, 10 ** 5) - base >= 2 * 4 * (10 ** 5 - 10) - 512


def test_stream_copy_rejects_bad_arguments_before_any_gpu_call(sss):
    L = sss.lib()
    v = ctypes.c_void_p(0x1000)
    assert L.sss_stream_copy(None, v, 64, None) == sss.ERR_INVALID
    assert L.sss_stream_copy(v, None, 64, None) == sss.ERR_INVALID
    assert L.sss_stream_copy(ctypes.c_void_p(0x1004), v, 64, None) == sss.ERR_INVALID
    assert L.sss_stream_copy(v, ctypes.c_void_p(0x1008), 64, None) == sss.ERR_INVALID
    assert L.sss_stream_copy(v, v, 40, None) == sss.ERR_INVALID
    assert L.sss_stream_copy(v, ctypes.c_void_p(0x2000), 0, None) == sss.OK   # nothing to launch


def test_sghmc_rejects_bad_arguments(sss):
    L = sss.lib()
    o = sss.SghmcOpts(0.01, 0.1, 100.0, 0.995, 0, 1, 0, 0)
    v = ctypes.c_void_p(0x1000)
    assert L.sss_sghmc_step(None, v, v, v, None, None, 10, ctypes.byref(o), None, None) == sss.ERR_INVALID
    assert L.sss_sghmc_step(v, v, v, v, None, None, 0, ctypes.byref(o), None, None) == sss.ERR_INVALID
    ob = sss.SghmcOpts(0.01, 0.1, 100.0, 0.995, 1, 1, 0, 0)
    assert L.sss_sghmc_step(v, v, v, v, None, None, 10, ctypes.byref(ob), None, None) == sss.ERR_INVALID
    bad = sss.SghmcOpts(-1.0, 0.1, 100.0, 0.995, 0, 1, 0, 0)
    assert L.sss_sghmc_step(v, v, v, v, None, None, 10, ctypes.byref(bad), None, None) == sss.ERR_INVALID
    ad = sss.Adam()
    ad.t = 0
    assert L.sss_sghmc_step(v, v, v, v, None, None, 10, ctypes.byref(o), ctypes.byref(ad), None) == sss.ERR_INVALID


def test_regularise_rejects_bad_arguments(sss):
    L = sss.lib()
    v = ctypes.c_void_p(0x1000)
    assert L.sss_regularise(None, v, 10, 0.1, 0.1, None, None, None, None) == sss.ERR_INVALID
    assert L.sss_regularise(v, v, 0, 0.1, 0.1, None, None, None, None) == sss.ERR_INVALID
    assert L.sss_regularise(v, v, 10, -0.1, 0.1, None, None, None, None) == sss.ERR_INVALID
    assert L.sss_regularise(v, v, 10, 0.1, float("nan"), None, None, None, None) == sss.ERR_INVALID


def test_records_layout_matches_decoder():
    from tests._util import REC_DTYPE
    assert REC_DTYPE.itemsize == 64
    assert REC_DTYPE.names[-2:] == ("entry", "ey")


def test_misaligned_workspaces_are_rejected(sss):
    """Workspaces are carved into 256-byte aligned parts: a misaligned ws is
    an argument error, found before anything is launched."""
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    p = _proj_struct(sss)
    b = sss.Bins(0x1000, 0x2000, 0x3000, 0x4000, None, None, None, 100, 0, 0)
    assert L.sss_bin_sort(ctypes.byref(p), cams, 1, 10, ctypes.byref(b), ctypes.c_void_p(0x9010), 10 ** 9,
                          None) == sss.ERR_INVALID
    assert b"aligned" in L.sss_last_error()
    opts = sss.render_opts()
    scene = _scene_struct(sss)
    g = sss.Grads(0, 0, 0, 0, 0, 0, 0, 0)
    assert L.sss_render_bwd(ctypes.byref(scene), ctypes.byref(p), ctypes.byref(b), cams, 1, ctypes.byref(opts), 0, 0,
                            ctypes.c_void_p(0x6000), ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000), None, None,
                            ctypes.byref(g), ctypes.c_void_p(0x9080), 10 ** 9, None) == sss.ERR_INVALID
    assert b"aligned" in L.sss_last_error()


def test_misaligned_scene_arrays_are_rejected(sss):
    """quats and SH rows are read with 16-byte loads: a scene whose quats or
    sh pointer is not 16-byte aligned is an argument error."""
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    opts = sss.render_opts()
    for idx in (2, 5):                                   # quats, sh
        scene = _scene_struct(sss)
        ptrs = [scene.means, scene.scales, scene.quats, scene.nu, scene.opacity, scene.sh]
        ptrs[idx] = ptrs[idx] + 4
        scene = sss.Scene(10, 0, 0, *[ctypes.c_void_p(q) for q in ptrs])
        p = _proj_struct(sss)
        assert L.sss_project(ctypes.byref(scene), cams, 1, ctypes.byref(opts), ctypes.byref(p), None) == sss.ERR_INVALID
        assert b"16-byte" in L.sss_last_error()


def test_binding_export_list_is_the_header(sss):
    """sss.EXPORTS (checked when the binding loads the library) lists exactly
    the functions include/sss.h declares."""
    assert sorted(sss.EXPORTS) == declared_functions()


def test_noalloc_rejects_bad_arguments_and_oversize_before_any_gpu_call(sss):
    """sss_render_bwd_noalloc checks its arguments, then the workspace the
    call needs against the array the library holds, before it looks up that
    array's device address: both errors come back on a machine without a
    GPU."""
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    opts = sss.render_opts()
    p = _proj_struct(sss)
    b = sss.Bins(0x1000, 0x2000, 0x3000, 0x4000, None, None, None, 100, 0, 0)
    g = sss.Grads(0, 0, 0, 0, 0, 0, 0, 0)

    def call(scene, mode):
        return L.sss_render_bwd_noalloc(ctypes.byref(scene), ctypes.byref(p), ctypes.byref(b), cams, 1,
                                        ctypes.byref(opts), mode, 0, ctypes.c_void_p(0x6000),
                                        ctypes.c_void_p(0x7000), ctypes.c_void_p(0x8000), None, None,
                                        ctypes.byref(g), None)

    assert call(_scene_struct(sss), 7) == sss.ERR_INVALID
    assert b"sss_render_bwd_noalloc" in L.sss_last_error()
    assert call(_scene_struct(sss, null=1), 0) == sss.ERR_INVALID
    # 1.5M entries need 1.5M x 96 B of per-entry sums: more than 128 MiB
    big = _scene_struct(sss, n=1_500_000)
    assert L.sss_render_bwd_workspace(1_500_000, 12) > (128 << 20)
    assert call(big, 0) == sss.ERR_INVALID
    assert b"SSS_NOALLOC_WORKSPACE_BYTES" in L.sss_last_error()


def test_project_rejects_misaligned_entries(sss):
    """Entries are 128-byte lines read with 16-byte loads: a pointer that is
    not 16-byte aligned is an argument error."""
    L = sss.lib()
    cams = sss.camera_array([scenes.ring_camera(64, 48)])
    scene = _scene_struct(sss)
    p = sss.Proj(0x2008, 0x3000, 0x5000)
    assert L.sss_project(ctypes.byref(scene), cams, 1, ctypes.byref(sss.render_opts()), ctypes.byref(p),
                         None) == sss.ERR_INVALID
    assert b"16-byte" in L.sss_last_error()


def test_struct_layouts_match_the_header(sss, tmp_path):
    """Every struct the binding passes has the size and field offsets the C
    compiler gives the header's declaration."""
    import subprocess
    structs = {"sss_scene_t": sss.Scene, "sss_grads_t": sss.Grads, "sss_camera_t": sss.Camera,
               "sss_render_opts_t": sss.RenderOpts, "sss_proj_t": sss.Proj, "sss_bins_t": sss.Bins,
               "sss_sghmc_opts_t": sss.SghmcOpts, "sss_adam_array_t": sss.AdamArray, "sss_adam_t": sss.Adam,
               "sss_step_t": sss.Step, "sss_relocate_opts_t": sss.RelocateOpts, "sss_state_t": sss.StateArray,
               "sss_kernel_time_t": sss.KernelTime}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sss.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
