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


def test_struct_layout_matches_c_compiler(tmp_path):
    """The binding's structures have the sizes and field offsets the C compiler
    gives the header's structures."""
    import subprocess
    fields = {"vm3dgs_options": ["img_w", "flags", "stream_render", "stream_copy", "pair_capacity", "lod_scale_up", "lod_builder"],
              "vm3dgs_camera": ["view", "cam_pos", "fx", "znear"],
              "vm3dgs_stats": ["candidates", "prefetched", "fallbacks", "render_gaussians", "blend_alphas", "ms_visibility",
                               "ms_total"],
              "vm3dgs_scene": ["n", "sh"],
              "vm3dgs_frame_out": ["requests", "n_requests", "missing", "n_missing", "stats"],
              "vm3dgs_prefetch_opts": ["n_clusters", "budget_pages", "logit_threshold", "center", "extent"],
              "vm3dgs_dataset": ["cams", "path_frames", "n_paths"],
              "vm3dgs_train_opts": ["steps", "batch", "lr", "seed", "proposal_factor", "log_every"],
              "vm3dgs_train_log": ["rows", "positive_rate", "loss_last", "ms_train", "n_losses", "losses"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vm3dgs.h"', "int main(void) {"]
    for s, fs in fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fs:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split("\n") if l)
    for s, fs in fields.items():
        cls = getattr(pkg, s)
        assert C.sizeof(cls) == int(out[s]), s
        for f in fs:
            assert getattr(cls, f).offset == int(out[f"{s}.{f}"]), (s, f)


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
