"""The C ABI library loads and exports every entry point of include/vm3dgs.h;
argument errors are reported before any device work (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2506_19415_amd as pkg
from paper_2506_19415_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vm3dgs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vm3dgs_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "vm3dgs_create" in names and "vm3dgs_frame" in names and "vm3dgs_render_full" in names
    L = C.CDLL(pkg.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_struct_sizes_match_header_layout():
    # the binding's structures must have the C layout (8-byte aligned pointers)
    assert C.sizeof(pkg.vm3dgs_options) == 72
    assert C.sizeof(pkg.vm3dgs_camera) == 96
    assert C.sizeof(pkg.vm3dgs_stats) == 112
    assert C.sizeof(pkg.vm3dgs_scene) == 48


def test_options_default():
    o = pkg.vm3dgs_options_default()
    assert (o.img_w, o.img_h, o.idbuf_w, o.idbuf_h, o.max_views) == (1920, 1080, 240, 135, 1)
    assert o.flags == pkg.VM3DGS_FLAG_LINKS and o.attr_format == 0 and o.lod_radius_px == 32.0


def test_create_rejects_bad_arguments_without_device():
    sc = synth.scene_clusters(0, n_clusters=1, per_cluster=100)
    with pytest.raises(pkg.Vm3dgsError) as e:
        pkg.vm3dgs_create(sc, 0, 8)
    assert e.value.code == -1
    with pytest.raises(pkg.Vm3dgsError) as e:
        pkg.vm3dgs_create(sc, 256, 0)
    assert e.value.code == -1
    with pytest.raises(pkg.Vm3dgsError) as e:
        pkg.vm3dgs_create(sc, 100, 8, lod_levels=2)   # 100 is not divisible by 8
    assert e.value.code == -1
    with pytest.raises(pkg.Vm3dgsError) as e:
        pkg.vm3dgs_create(sc, 256, 8, lod_levels=4)
    assert e.value.code == -1
    o = pkg.vm3dgs_options_default()
    o.max_views = 0
    with pytest.raises(pkg.Vm3dgsError):
        pkg.vm3dgs_create(sc, 256, 8, 1, o)
    o = pkg.vm3dgs_options_default()
    o.attr_format = 7
    with pytest.raises(pkg.Vm3dgsError):
        pkg.vm3dgs_create(sc, 256, 8, 1, o)


def test_null_handles_are_safe():
    L = pkg.lib()
    L.vm3dgs_destroy(None)
    assert L.vm3dgs_sync(None) == -1
    assert L.vm3dgs_frame(None, None, 0, None, None) == -1
    assert L.vm3dgs_debug_get(None, b"info", None, 0) == -1
    empty = pkg.vm3dgs_scene(0, None, None, None, None, None)
    h = C.c_void_p()
    assert L.vm3dgs_pages_build(C.byref(empty), 256, 1, None, C.byref(h)) == -1
