"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  It loads ``oracle/liboracle.so`` (built by
``oracle/build.py``) and never touches the product library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class _Cam(C.Structure):
    _fields_ = [("view", C.c_float * 16), ("cam_pos", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("znear", C.c_float)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401
            _b.build()
        L = C.CDLL(path)
        L.or_vm_exp.restype = C.c_float
        L.or_vm_exp.argtypes = [C.c_float]
        L.or_sh_basis.restype = C.c_double
        L.or_sh_basis.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.or_round_f16.restype = C.c_float
        L.or_round_f16.argtypes = [C.c_float]
        L.or_round_bf16.restype = C.c_float
        L.or_round_bf16.argtypes = [C.c_float]
        L.or_scene_build.restype = C.c_void_p
        L.or_scene_build.argtypes = [C.POINTER(_Scene), C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                     C.c_float, C.c_int]
        L.or_kmeans_page.restype = C.c_int
        L.or_kmeans_page.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p]
        L.or_scene_free.argtypes = [C.c_void_p]
        L.or_scene_get.restype = C.c_int64
        L.or_scene_get.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64]
        L.or_vm_create.restype = C.c_void_p
        L.or_vm_create.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_float, C.c_float]
        L.or_vm_free.argtypes = [C.c_void_p]
        L.or_vm_frame.argtypes = [C.c_void_p, C.POINTER(_Cam), C.c_int, C.c_void_p]
        L.or_vm_visibility.argtypes = [C.c_void_p, C.POINTER(_Cam), C.c_int, C.c_int]
        L.or_render_full.argtypes = [C.c_void_p, C.POINTER(_Cam), C.c_int, C.c_void_p]
        L.or_vm_get.restype = C.c_int64
        L.or_vm_get.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64]
        L.or_vm_set_async.argtypes = [C.c_void_p, C.c_int]
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = C.c_int
        L.or_merge_children.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p]
        L.or_merge_children_d.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_void_p]
        L.or_lod_level.restype = C.c_int
        L.or_lod_level.argtypes = [C.c_float, C.c_float, C.c_float, C.c_float, C.c_int]
        L.or_lod_control_trace.argtypes = [C.c_int, C.c_int, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        for nm in ("or_vm_exp_n", "or_round_f16_n", "or_round_bf16_n"):
            getattr(L, nm).argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.or_vm_pagetable.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.or_vm_set_force_all.argtypes = [C.c_void_p, C.c_int]
        L.or_vm_set_support_box.argtypes = [C.c_void_p, C.c_int]
        L.or_vm_set_adaptive_lod.argtypes = [C.c_void_p, C.c_int]
        L.or_vm_render_fp64.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(_Cam), C.c_int, C.c_void_p]
        L.or_vm_set_prefetch.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_float, C.c_int, C.c_void_p, C.c_float]
        L.or_vm_features.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.or_vm_frame_prefetch.argtypes = [C.c_void_p, C.POINTER(_Cam), C.c_int, C.c_void_p, C.c_void_p]
        if hasattr(L, "or_mlp_forward"):
            _bind_mlp(L)
        _LIB = L
    return _LIB


def _bind_mlp(L):
    d = C.c_void_p
    L.or_mlp_n_params.restype = C.c_int64
    L.or_mlp_n_params.argtypes = [C.c_int, d]
    L.or_mlp_forward.argtypes = [C.c_int, C.c_int, d, d, d, C.c_int, d]
    L.or_mlp_backward.argtypes = [C.c_int, C.c_int, d, d, d, d, C.c_int, d, d]
    L.or_mlp_backward.restype = C.c_double
    L.or_adam.argtypes = [C.c_int64, d, d, d, d, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]


def _cam(c) -> _Cam:
    out = _Cam()
    v = np.ascontiguousarray(c.view, dtype=np.float32).reshape(16)
    for i in range(16):
        out.view[i] = float(v[i])
    for i in range(3):
        out.cam_pos[i] = float(c.cam_pos[i])
    out.fx, out.fy, out.cx, out.cy, out.znear = float(c.fx), float(c.fy), float(c.cx), float(c.cy), float(c.znear)
    return out


def cams_array(cams):
    arr = (_Cam * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = _cam(c)
    return arr


def vm_exp(x: float) -> float:
    return lib().or_vm_exp(float(x))


def _vec(fn, x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    getattr(lib(), fn)(x.ctypes.data, y.ctypes.data, x.size)
    return y


def vm_exp_n(x):
    return _vec("or_vm_exp_n", x)


def round_f16_n(x):
    return _vec("or_round_f16_n", x)


def round_bf16_n(x):
    return _vec("or_round_bf16_n", x)


def sh_basis(k, x, y, z) -> float:
    return lib().or_sh_basis(int(k), float(x), float(y), float(z))


def round_f16(x: float) -> float:
    return lib().or_round_f16(float(x))


def round_bf16(x: float) -> float:
    return lib().or_round_bf16(float(x))


def kmeans_page(records, k, scale_up=1.0):
    """The k parents of one page's level from its records ([n][59] float32)
    by the k-means builder; returns (parents [k][59], cluster of each record
    (-1 for padding), Lloyd iterations run)."""
    r = np.ascontiguousarray(records, dtype=np.float32)
    out = np.zeros((k, 59), np.float32)
    assign = np.zeros(len(r), np.int32)
    it = lib().or_kmeans_page(r.ctypes.data, len(r), int(k), float(scale_up), out.ctypes.data, assign.ctypes.data)
    return out, assign, int(it)


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's splat loops and k-means LOD levels (n > 0
    sets); returns the count in use."""
    return int(lib().or_set_threads(int(n)))


def merge_children(rec: np.ndarray, scale_up: float = 1.0) -> np.ndarray:
    """Stored (float32) parent record of the children rec [k][59]."""
    rec = np.ascontiguousarray(rec, dtype=np.float32)
    out = np.zeros(59, dtype=np.float32)
    lib().or_merge_children(rec.ctypes.data, rec.shape[0], float(scale_up), out.ctypes.data)
    return out


def merge_children_d(rec: np.ndarray, scale_up: float = 1.0) -> np.ndarray:
    """Parent record of the children rec [k][59] in double, before rounding."""
    rec = np.ascontiguousarray(rec, dtype=np.float32)
    out = np.zeros(59, dtype=np.float64)
    lib().or_merge_children_d(rec.ctypes.data, rec.shape[0], float(scale_up), out.ctypes.data)
    return out


def lod_level(fy: float, radius: float, depth: float, tau: float, levels: int) -> int:
    return int(lib().or_lod_level(float(fy), float(radius), float(depth), float(tau), int(levels)))


def lod_control_trace(S: int, tau0: float, req_slots, n_missing, n_coarse):
    """The memory-use controller over a sequence of frames from a fresh
    state: (tau, step) after each frame, float32 arrays."""
    rs = np.ascontiguousarray(req_slots, dtype=np.int32)
    nm = np.ascontiguousarray(n_missing, dtype=np.int32)
    nc = np.ascontiguousarray(n_coarse, dtype=np.int32)
    n = rs.shape[0]
    assert nm.shape[0] == n and nc.shape[0] == n
    tau = np.zeros(n, np.float32)
    step = np.zeros(n, np.float32)
    lib().or_lod_control_trace(n, int(S), float(tau0), rs.ctypes.data, nm.ctypes.data, nc.ctypes.data,
                               tau.ctypes.data, step.ctypes.data)
    return tau, step


_SCENE_DT = {"perm": np.int64, "attr0": np.float32, "attr1": np.float32, "attr2": np.float32,
             "spheres": np.float32, "cell_box": np.float32, "cell_page": np.int32,
             "cell_start": np.int32, "link_start": np.int32, "link_dst": np.int32,
             "n_pages": np.int64, "n_cells": np.int64, "n_links": np.int64, "lo": np.float64}

_VM_DT = {"lod": np.float32, "pf_keys": np.uint64, "pf_x": np.float32, "pf_counts": np.int64, "frame": np.int64, "cand": np.uint8, "idbuf": np.uint64, "req_direct": np.uint32,
          "req_link": np.uint32, "page_level": np.int8, "req_page": np.int32, "req_level": np.int8,
          "req_class": np.uint8, "slot_level": np.int8, "last_used": np.int32, "sub_vpage": np.int32,
          "sub_last_used": np.int32, "v2p": np.int32, "copies": np.int64, "copy_id": np.int32,
          "missing": np.int32, "counts": np.int64, "render_list": np.int32, "pp_float": np.float32,
          "pp_int": np.int32, "n_pairs": np.int64, "keys": np.uint64, "vals": np.uint32,
          "ranges": np.uint32, "image": np.float32, "final_T": np.float32, "contrib": np.int64,
          "visits": np.int64}


class OracleScene:
    """Create-time data built by the oracle (Morton pages, proxy, links, LOD)."""

    def __init__(self, scene, page_size, lod_levels=1, cell_m=0.5, link_sigma=2.0, attr_format=0, lod_scale_up=1.0,
                 lod_builder=0):
        self._keep = [np.ascontiguousarray(a, dtype=np.float32) for a in
                      (scene.means, scene.scales, scene.quats, scene.opacity, scene.sh)]
        s = _Scene(scene.n, *[a.ctypes.data for a in self._keep])
        self.ptr = lib().or_scene_build(C.byref(s), int(page_size), int(lod_levels), float(cell_m),
                                        float(link_sigma), int(attr_format), float(lod_scale_up),
                                        int(lod_builder))
        if not self.ptr:
            raise ValueError("oracle: invalid scene parameters")
        self.page_size = page_size
        self.lod_levels = lod_levels
        self.n_pages = int(self.get("n_pages")[0])

    def get(self, name):
        n = lib().or_scene_get(self.ptr, name.encode(), None, 0)
        if n < 0:
            raise KeyError(name)
        out = np.empty(n // np.dtype(_SCENE_DT[name]).itemsize, dtype=_SCENE_DT[name])
        lib().or_scene_get(self.ptr, name.encode(), out.ctypes.data, n)
        return out

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().or_scene_free(self.ptr)
            self.ptr = None


class OracleVM:
    """Per-frame oracle state: page table over ``pool_pages`` physical pages."""

    def __init__(self, oscene: OracleScene, pool_pages, img, idbuf, copy_budget=0, use_links=True,
                 lod_radius_px=32.0, guard_px=32.0, support_box=False):
        self.scene = oscene
        self.W, self.H = img
        self.Wv, self.Hv = idbuf
        self.TX, self.TY = (self.W + 15) // 16, (self.H + 15) // 16
        self.ptr = lib().or_vm_create(oscene.ptr, int(pool_pages), int(copy_budget), int(bool(use_links)),
                                      self.W, self.H, self.Wv, self.Hv, float(lod_radius_px), float(guard_px))
        if not self.ptr:
            raise ValueError("oracle: invalid VM parameters")
        if support_box:
            self.set_support_box(True)

    def frame(self, cams, tile_mask=None):
        arr = cams_array(cams)
        m = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        lib().or_vm_frame(self.ptr, arr, len(cams), None if m is None else m.ctypes.data)

    def visibility(self, cams, brute_force=False):
        arr = cams_array(cams)
        lib().or_vm_visibility(self.ptr, arr, len(cams), int(bool(brute_force)))

    def render_full(self, cams, tile_mask=None):
        arr = cams_array(cams)
        m = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        lib().or_render_full(self.ptr, arr, len(cams), None if m is None else m.ctypes.data)

    def pagetable(self, pages, levels=None):
        p = np.ascontiguousarray(pages, dtype=np.int32)
        lv = None if levels is None else np.ascontiguousarray(levels, dtype=np.int8)
        lib().or_vm_pagetable(self.ptr, len(p), p.ctypes.data, None if lv is None else lv.ctypes.data)

    def set_force_all(self, on=True):
        lib().or_vm_set_force_all(self.ptr, int(bool(on)))

    def set_prefetch(self, n_clusters, hist_bins, logit_threshold, budget_pages, center, extent):
        c = np.ascontiguousarray(center, dtype=np.float32)
        self.pf_dims = (int(n_clusters), int(hist_bins))
        assert lib().or_vm_set_prefetch(self.ptr, int(n_clusters), int(hist_bins), float(logit_threshold),
                                        int(budget_pages), c.ctypes.data, float(extent)) == 0

    def features(self, view=0):
        x = np.zeros(28 + self.pf_dims[1], np.float32)
        lib().or_vm_features(self.ptr, int(view), x.ctypes.data)
        return x

    def frame_prefetch(self, cams, logits, tile_mask=None):
        arr = cams_array(cams)
        z = np.ascontiguousarray(logits, dtype=np.float32)
        assert z.shape == (len(cams), self.pf_dims[0])
        m = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
        lib().or_vm_frame_prefetch(self.ptr, arr, len(cams), z.ctypes.data, None if m is None else m.ctypes.data)

    def render_fp64(self, src_scene, cams):
        """FP64 splat of the last frame's render set with the attributes of
        src_scene (an OracleScene of the same pages)."""
        arr = cams_array(cams)
        img = np.zeros((len(cams), self.H, self.W, 3), np.float64)
        lib().or_vm_render_fp64(self.ptr, src_scene.ptr, arr, len(cams), img.ctypes.data)
        return img

    def set_adaptive_lod(self, on=True):
        lib().or_vm_set_adaptive_lod(self.ptr, int(bool(on)))

    def set_support_box(self, on=True):
        """Cut each 3-sigma tile rectangle to the Gaussian's support box (the
        pixels where a term can pass the alpha test).  Off by default; the
        image is the same either way, and with it on the pair list is that of
        a renderer that makes this cut."""
        lib().or_vm_set_support_box(self.ptr, int(bool(on)))

    def get(self, name):
        n = lib().or_vm_get(self.ptr, name.encode(), None, 0)
        if n < 0:
            raise KeyError(name)
        dt = np.dtype(_VM_DT[name])
        out = np.empty(n // dt.itemsize, dtype=dt)
        if n > 0:
            lib().or_vm_get(self.ptr, name.encode(), out.ctypes.data, n)
        return out

    def counts(self):
        c = self.get("counts")
        return dict(zip(["requests", "hits", "misses", "evictions", "copies", "missing",
                         "render_pages", "render_gaussians", "fallbacks"], [int(x) for x in c]))

    def set_async(self, on=True):
        """Streaming: the frame renders what was resident when it started and
        its copies land for the next frame."""
        lib().or_vm_set_async(self.ptr, int(bool(on)))

    def image(self, n_views=1):
        return self.get("image").reshape(n_views, self.H, self.W, 3)

    def __del__(self):
        if getattr(self, "ptr", None):
            lib().or_vm_free(self.ptr)
            self.ptr = None


# ---------------------------------------------------------------- prefetch network
def mlp_n_params(dims):
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    return int(lib().or_mlp_n_params(len(dims) - 1, dm.ctypes.data))


def mlp_forward(params, dims, x, bf16=True):
    """Logits [B][d_L] in double."""
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float32)
    B = xx.shape[0]
    z = np.zeros((B, dims[-1]), np.float64)
    lib().or_mlp_forward(B, len(dims) - 1, dm.ctypes.data, p.ctypes.data, xx.ctypes.data, int(bool(bf16)),
                         z.ctypes.data)
    return z


def mlp_backward(params, dims, x, y, bf16=True):
    """(loss, grad in the parameter layout, logits)."""
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.float32)
    xx = np.ascontiguousarray(x, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    B = xx.shape[0]
    g = np.zeros(p.size, np.float64)
    z = np.zeros((B, dims[-1]), np.float64)
    loss = lib().or_mlp_backward(B, len(dims) - 1, dm.ctypes.data, p.ctypes.data, xx.ctypes.data, yy.ctypes.data,
                                 int(bool(bf16)), g.ctypes.data, z.ctypes.data)
    return loss, g, z


def adam(w, m, v, g, lr, b1, b2, eps, t):
    """One Adam step on float32 arrays w, m, v (in place)."""
    for a in (w, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    gg = np.ascontiguousarray(g, dtype=np.float64)
    lib().or_adam(w.size, w.ctypes.data, m.ctypes.data, v.ctypes.data, gg.ctypes.data, lr, b1, b2, eps, int(t))
