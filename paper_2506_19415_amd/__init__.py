"""Python binding of the MI355X virtual-memory 3DGS library (libvm3dgs.so).

Thin ctypes layer over include/vm3dgs.h: the functions below have the C
names and only marshal arguments; every step of a frame runs in the HIP
kernels of the shared library.  PyTorch is used for device memory (the
output image) only.  When the shared library is missing this module raises
at import of the library (no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvm3dgs.so")

VM3DGS_FLAG_LINKS = 1
VM3DGS_FLAG_FULL_SCENE_COPY = 2
VM3DGS_FLAG_BLEND_STATS = 4
VM3DGS_FLAG_SIGMA3_TILES = 8
VM3DGS_FLAG_ADAPTIVE_LOD = 16
VM3DGS_FLAG_ASYNC_MISSES = 32
VM3DGS_NOALLOC_MAX_PAIRS = 7864320

_ERRORS = {-1: "INVALID_ARG", -2: "HOST_OOM", -3: "DEVICE_OOM", -4: "HIP", -5: "STATE", -6: "CAPACITY"}


class Vm3dgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vm3dgs error {code} ({_ERRORS.get(code, '?')}): {msg}")
        self.code = code


class vm3dgs_scene(C.Structure):
    _fields_ = [("n", C.c_uint64), ("means", C.c_void_p), ("scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity", C.c_void_p), ("sh", C.c_void_p)]


class vm3dgs_options(C.Structure):
    _fields_ = [("img_w", C.c_uint32), ("img_h", C.c_uint32), ("idbuf_w", C.c_uint32), ("idbuf_h", C.c_uint32),
                ("max_views", C.c_uint32), ("attr_format", C.c_uint32), ("copy_budget_pages", C.c_uint32),
                ("idbuf_guard_px", C.c_float), ("proxy_cell_m", C.c_float), ("link_sigma", C.c_float),
                ("lod_radius_px", C.c_float), ("flags", C.c_uint32), ("stream_render", C.c_void_p),
                ("stream_copy", C.c_void_p), ("pair_capacity", C.c_uint64), ("lod_scale_up", C.c_float),
                ("lod_builder", C.c_uint32)]


class vm3dgs_camera(C.Structure):
    _fields_ = [("view", C.c_float * 16), ("cam_pos", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("znear", C.c_float)]


class vm3dgs_prefetch_opts(C.Structure):
    _fields_ = [("n_clusters", C.c_uint32), ("hist_bins", C.c_uint32), ("budget_pages", C.c_uint32),
                ("logit_threshold", C.c_float), ("center", C.c_float * 3), ("extent", C.c_float)]


class vm3dgs_stats(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("candidates", "requested", "direct", "linked", "hits", "misses",
                                           "evictions", "missing", "copies", "render_pages", "pool_pages_used",
                                           "prefetched", "fallbacks")] + \
               [(n, C.c_uint64) for n in ("render_gaussians", "visible_gaussians", "pairs", "bytes_copied",
                                           "blend_evals", "blend_alphas")] + \
               [(n, C.c_float) for n in ("ms_visibility", "ms_pagetable", "ms_copy", "ms_preprocess", "ms_sort",
                                          "ms_blend", "ms_total", "lod_radius_px")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vm3dgs_dataset(C.Structure):
    _fields_ = [("cams", C.c_void_p), ("path_frames", C.c_void_p), ("n_paths", C.c_uint32)]


class vm3dgs_train_opts(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("batch", C.c_uint32), ("lr", C.c_float), ("seed", C.c_uint64),
                ("proposal_factor", C.c_float), ("log_every", C.c_uint32)]


class vm3dgs_train_log(C.Structure):
    _fields_ = [("rows", C.c_uint64), ("positive_rate", C.c_float), ("loss_first", C.c_float),
                ("loss_last", C.c_float), ("logit_threshold", C.c_float), ("ms_collect", C.c_float),
                ("ms_train", C.c_float), ("n_losses", C.c_uint32), ("losses", C.c_float * 64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "losses"}
        d["losses"] = [float(self.losses[i]) for i in range(self.n_losses)]
        return d


class vm3dgs_frame_out(C.Structure):
    _fields_ = [("requests", C.POINTER(C.c_int32)), ("request_level", C.POINTER(C.c_int8)),
                ("n_requests", C.c_uint32), ("missing", C.POINTER(C.c_int32)), ("n_missing", C.c_uint32),
                ("stats", vm3dgs_stats)]


_lib = None


def lib():
    """Load libvm3dgs.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_19415_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.vm3dgs_options_default.argtypes = [C.POINTER(vm3dgs_options)]
        L.vm3dgs_create.argtypes = [C.POINTER(vm3dgs_scene), C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.POINTER(vm3dgs_options), C.POINTER(C.c_void_p)]
        L.vm3dgs_create.restype = C.c_int32
        L.vm3dgs_frame.argtypes = [C.c_void_p, C.POINTER(vm3dgs_camera), C.c_uint32, C.c_void_p,
                                   C.POINTER(vm3dgs_frame_out)]
        L.vm3dgs_frame.restype = C.c_int32
        L.vm3dgs_frame_noalloc.argtypes = [C.c_void_p, C.POINTER(vm3dgs_camera), C.c_uint32, C.c_void_p,
                                           C.POINTER(vm3dgs_frame_out)]
        L.vm3dgs_frame_noalloc.restype = C.c_int32
        L.vm3dgs_render_full.argtypes = [C.c_void_p, C.POINTER(vm3dgs_camera), C.c_uint32, C.c_void_p,
                                         C.POINTER(vm3dgs_stats)]
        L.vm3dgs_render_full.restype = C.c_int32
        L.vm3dgs_debug_get.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64]
        L.vm3dgs_debug_get.restype = C.c_int64
        L.vm3dgs_set_flags.argtypes = [C.c_void_p, C.c_uint32]
        L.vm3dgs_set_flags.restype = C.c_int32
        L.vm3dgs_set_lod_radius.argtypes = [C.c_void_p, C.c_float]
        L.vm3dgs_set_lod_radius.restype = C.c_int32
        L.vm3dgs_sync.argtypes = [C.c_void_p]
        L.vm3dgs_sync.restype = C.c_int32
        L.vm3dgs_last_error.argtypes = [C.c_void_p]
        L.vm3dgs_last_error.restype = C.c_char_p
        L.vm3dgs_create_error.argtypes = []
        L.vm3dgs_create_error.restype = C.c_char_p
        L.vm3dgs_destroy.argtypes = [C.c_void_p]
        L.vm3dgs_pages_build.argtypes = [C.POINTER(vm3dgs_scene), C.c_uint32, C.c_uint32,
                                         C.POINTER(vm3dgs_options), C.POINTER(C.c_void_p)]
        L.vm3dgs_pages_build.restype = C.c_int32
        L.vm3dgs_pages_get.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64]
        L.vm3dgs_pages_get.restype = C.c_int64
        L.vm3dgs_pages_destroy.argtypes = [C.c_void_p]
        vp, u32 = C.c_void_p, C.c_uint32
        for name, args in [("vm3dgs_mlp_create", [vp, u32, u32, vp, C.POINTER(vp)]),
                           ("vm3dgs_mlp_set_params", [vp, vp, C.c_uint64]),
                           ("vm3dgs_mlp_get_state", [vp, vp, vp, vp, C.c_uint64, vp]),
                           ("vm3dgs_mlp_forward", [vp, vp, u32, vp]),
                           ("vm3dgs_mlp_gradient", [vp, vp, vp, u32, vp, vp]),
                           ("vm3dgs_mlp_train_step", [vp, vp, vp, u32, C.c_float, vp]),
                           ("vm3dgs_mlp_sync", [vp])]:
            getattr(L, name).argtypes = args
            getattr(L, name).restype = C.c_int32
        L.vm3dgs_mlp_create_error.argtypes = []
        L.vm3dgs_mlp_create_error.restype = C.c_char_p
        L.vm3dgs_mlp_last_error.argtypes = [vp]
        L.vm3dgs_mlp_last_error.restype = C.c_char_p
        L.vm3dgs_mlp_n_params.argtypes = [vp]
        L.vm3dgs_mlp_n_params.restype = C.c_uint64
        L.vm3dgs_mlp_destroy.argtypes = [vp]
        L.vm3dgs_reset.argtypes = [vp]
        L.vm3dgs_reset.restype = C.c_int32
        L.vm3dgs_set_prefetch.argtypes = [vp, vp, C.POINTER(vm3dgs_prefetch_opts)]
        L.vm3dgs_set_prefetch.restype = C.c_int32
        L.vm3dgs_prefetch_features.argtypes = [vp, u32, vp]
        L.vm3dgs_prefetch_features.restype = C.c_int32
        L.vm3dgs_prefetch_collect.argtypes = [vp, C.POINTER(vm3dgs_dataset), vp, vp, C.c_uint64,
                                              C.POINTER(C.c_uint64)]
        L.vm3dgs_prefetch_collect.restype = C.c_int32
        L.vm3dgs_prefetch_train.argtypes = [vp, C.POINTER(vm3dgs_dataset), C.POINTER(vm3dgs_train_opts),
                                            C.POINTER(vm3dgs_train_log)]
        L.vm3dgs_prefetch_train.restype = C.c_int32
        for name in ("vm3dgs_mlp_save", "vm3dgs_mlp_load", "vm3dgs_prefetch_load"):
            getattr(L, name).argtypes = [vp, C.c_char_p]
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


# ------------------------------------------------------------------ C names
def vm3dgs_options_default() -> vm3dgs_options:
    o = vm3dgs_options()
    lib().vm3dgs_options_default(C.byref(o))
    return o


def pack_cameras(cams):
    """The cameras as the C array vm3dgs_frame takes; the frame calls accept
    such an array in place of a list (a caller that renders the same cameras
    again, or times its frames, packs them once)."""
    return _cameras(cams)


def _cameras(cams):
    if isinstance(cams, C.Array) and cams._type_ is vm3dgs_camera:
        return cams
    arr = (vm3dgs_camera * len(cams))()
    for i, c in enumerate(cams):
        v = np.ascontiguousarray(c.view, dtype=np.float32).reshape(16)
        arr[i].view[:] = [float(x) for x in v]
        arr[i].cam_pos[:] = [float(x) for x in np.asarray(c.cam_pos, np.float32)]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy, arr[i].znear = (float(c.fx), float(c.fy), float(c.cx),
                                                                    float(c.cy), float(c.znear))
    return arr


def vm3dgs_create(scene, page_size, pool_pages, lod_levels=1, opts: vm3dgs_options = None):
    keep = [np.ascontiguousarray(a, dtype=np.float32) for a in
            (scene.means, scene.scales, scene.quats, scene.opacity, scene.sh)]
    s = vm3dgs_scene(scene.n, *[a.ctypes.data for a in keep])
    h = C.c_void_p()
    rc = lib().vm3dgs_create(C.byref(s), int(page_size), int(pool_pages), int(lod_levels),
                             None if opts is None else C.byref(opts), C.byref(h))
    if rc != 0:
        raise Vm3dgsError(rc, lib().vm3dgs_create_error().decode())
    return h


def _check(h, rc):
    if rc != 0:
        raise Vm3dgsError(rc, lib().vm3dgs_last_error(h).decode())


def vm3dgs_frame(h, cams, image_dev_ptr: int) -> vm3dgs_frame_out:
    out = vm3dgs_frame_out()
    arr = _cameras(cams)
    _check(h, lib().vm3dgs_frame(h, arr, len(cams), C.c_void_p(image_dev_ptr), C.byref(out)))
    return out


def vm3dgs_frame_noalloc(h, cams, image_dev_ptr: int) -> vm3dgs_frame_out:
    out = vm3dgs_frame_out()
    arr = _cameras(cams)
    _check(h, lib().vm3dgs_frame_noalloc(h, arr, len(cams), C.c_void_p(image_dev_ptr), C.byref(out)))
    return out


def vm3dgs_render_full(h, cams, image_dev_ptr: int) -> vm3dgs_stats:
    st = vm3dgs_stats()
    arr = _cameras(cams)
    _check(h, lib().vm3dgs_render_full(h, arr, len(cams), C.c_void_p(image_dev_ptr), C.byref(st)))
    return st


def vm3dgs_debug_get(h, name: str, dtype) -> np.ndarray:
    n = lib().vm3dgs_debug_get(h, name.encode(), None, 0)
    if n < 0:
        raise KeyError(name)
    dt = np.dtype(dtype)
    out = np.empty(n // dt.itemsize, dtype=dt)
    if n > 0 and lib().vm3dgs_debug_get(h, name.encode(), out.ctypes.data, n) < 0:
        raise Vm3dgsError(-4, "debug copy failed")
    return out


def vm3dgs_pages_build(scene, page_size, lod_levels=1, opts: vm3dgs_options = None):
    keep = [np.ascontiguousarray(a, dtype=np.float32) for a in
            (scene.means, scene.scales, scene.quats, scene.opacity, scene.sh)]
    s = vm3dgs_scene(scene.n, *[a.ctypes.data for a in keep])
    h = C.c_void_p()
    rc = lib().vm3dgs_pages_build(C.byref(s), int(page_size), int(lod_levels),
                                  None if opts is None else C.byref(opts), C.byref(h))
    if rc != 0:
        raise Vm3dgsError(rc, lib().vm3dgs_create_error().decode())
    return h


def vm3dgs_pages_get(h, name: str, dtype) -> np.ndarray:
    n = lib().vm3dgs_pages_get(h, name.encode(), None, 0)
    if n < 0:
        raise KeyError(name)
    dt = np.dtype(dtype)
    out = np.empty(n // dt.itemsize, dtype=dt)
    if n > 0:
        lib().vm3dgs_pages_get(h, name.encode(), out.ctypes.data, n)
    return out


def vm3dgs_pages_destroy(h):
    lib().vm3dgs_pages_destroy(h)


def vm3dgs_set_flags(h, flags: int):
    _check(h, lib().vm3dgs_set_flags(h, int(flags)))


def vm3dgs_set_lod_radius(h, tau_px: float):
    _check(h, lib().vm3dgs_set_lod_radius(h, float(tau_px)))


def vm3dgs_sync(h):
    _check(h, lib().vm3dgs_sync(h))


def vm3dgs_destroy(h):
    lib().vm3dgs_destroy(h)


# ------------------------------------------------------------------ convenience
class Renderer:
    """Owns one library context and a device image buffer (torch tensor)."""

    def __init__(self, scene, page_size, pool_pages, lod_levels=1, img=(1920, 1080), idbuf=(240, 135),
                 max_views=1, attr_format=0, cell=1.0, link_sigma=2.0, lod_radius_px=32.0, links=True,
                 full_scene=False, copy_budget=0, pair_capacity=0, guard_px=32.0, lod_scale_up=1.0,
                 lod_builder=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Renderer needs a HIP device")
        o = vm3dgs_options_default()
        o.img_w, o.img_h = img
        o.idbuf_w, o.idbuf_h = idbuf
        o.max_views = max_views
        o.attr_format = attr_format
        o.copy_budget_pages = copy_budget
        o.idbuf_guard_px = guard_px
        o.proxy_cell_m, o.link_sigma, o.lod_radius_px = cell, link_sigma, lod_radius_px
        o.flags = (VM3DGS_FLAG_LINKS if links else 0) | (VM3DGS_FLAG_FULL_SCENE_COPY if full_scene else 0)
        o.pair_capacity = pair_capacity
        o.lod_scale_up = lod_scale_up
        o.lod_builder = lod_builder
        self.opts = o
        self.W, self.H = img
        self.h = vm3dgs_create(scene, page_size, pool_pages, lod_levels, o)
        self.image = torch.empty((max_views, self.H, self.W, 3), dtype=torch.float32, device="cuda")

    # The library renders on streams of its own and returns once the image is
    # complete; before it overwrites the image, torch's pending work (which
    # may still read the previous image) is waited for (a query first: an idle
    # stream costs no wait).
    @staticmethod
    def _torch_idle():
        import torch
        s = torch.cuda.current_stream()
        if not s.query():
            s.synchronize()

    def frame(self, cams):
        self._torch_idle()
        out = vm3dgs_frame(self.h, cams, self.image.data_ptr())
        return self.image[:len(cams)], out

    def frame_noalloc(self, cams):
        """vm3dgs_frame_noalloc: the same frame with the pair buffers in the
        library's fixed device scratch (nothing allocated)."""
        self._torch_idle()
        out = vm3dgs_frame_noalloc(self.h, cams, self.image.data_ptr())
        return self.image[:len(cams)], out

    def render_full(self, cams):
        self._torch_idle()
        st = vm3dgs_render_full(self.h, cams, self.image.data_ptr())
        return self.image[:len(cams)], st

    def set_prefetch(self, net, n_clusters, hist_bins, logit_threshold, budget_pages, center, extent):
        """Attach the learned prefetch stage (net: an Mlp, or None to keep
        only the pose history for vm3dgs_prefetch_features)."""
        o = vm3dgs_prefetch_opts()
        o.n_clusters, o.hist_bins, o.budget_pages = int(n_clusters), int(hist_bins), int(budget_pages)
        o.logit_threshold = float(logit_threshold)
        o.center[:] = [float(v) for v in center]
        o.extent = float(extent)
        rc = lib().vm3dgs_set_prefetch(self.h, net.h if net is not None else None, C.byref(o))
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_last_error(self.h).decode())
        self.pf_net = net
        self.pf_opts = o
        self.pf_width = 28 + int(hist_bins)

    def reset(self):
        rc = lib().vm3dgs_reset(self.h)
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_last_error(self.h).decode())

    def _dataset(self, paths):
        """A vm3dgs_dataset of camera paths (one view per frame); the arrays
        it points to are returned with it and must outlive the call."""
        cams = [c for p in paths for c in p]
        arr = _cameras(cams)
        frames = (C.c_uint32 * len(paths))(*[len(p) for p in paths])
        return vm3dgs_dataset(C.cast(arr, C.c_void_p), C.cast(frames, C.c_void_p), len(paths)), (arr, frames)

    def prefetch_collect(self, paths):
        """vm3dgs_prefetch_collect: feature and label rows of the paths."""
        ds, keep = self._dataset(paths)
        rows = sum(max(len(p) - 1, 0) for p in paths)
        o = self.pf_opts
        X = np.zeros((rows, 28 + o.hist_bins), np.float32)
        Y = np.zeros((rows, o.n_clusters), np.float32)
        n = C.c_uint64()
        rc = lib().vm3dgs_prefetch_collect(self.h, C.byref(ds), X.ctypes.data, Y.ctypes.data, rows, C.byref(n))
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_last_error(self.h).decode())
        return X[:n.value], Y[:n.value]

    def prefetch_train(self, paths, steps, batch=256, lr=1e-3, seed=0, proposal_factor=0.0, log_every=0):
        """vm3dgs_prefetch_train on the attached network; returns the log."""
        ds, keep = self._dataset(paths)
        t = vm3dgs_train_opts(int(steps), int(batch), float(lr), int(seed), float(proposal_factor), int(log_every))
        log_ = vm3dgs_train_log()
        rc = lib().vm3dgs_prefetch_train(self.h, C.byref(ds), C.byref(t), C.byref(log_))
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_last_error(self.h).decode())
        self.pf_opts.logit_threshold = log_.logit_threshold
        return log_.as_dict()

    def prefetch_load(self, path):
        rc = lib().vm3dgs_prefetch_load(self.h, str(path).encode())
        if rc != 0:
            raise Vm3dgsError(rc, "vm3dgs_prefetch_load failed")

    def prefetch_features(self, n_views=1):
        x = np.zeros((n_views, self.pf_width), np.float32)
        rc = lib().vm3dgs_prefetch_features(self.h, int(n_views), x.ctypes.data)
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_last_error(self.h).decode())
        return x

    def set_flags(self, flags):
        vm3dgs_set_flags(self.h, flags)
        self.opts.flags = (self.opts.flags & VM3DGS_FLAG_FULL_SCENE_COPY) | (flags & ~VM3DGS_FLAG_FULL_SCENE_COPY)

    def set_lod_radius(self, tau_px):
        vm3dgs_set_lod_radius(self.h, tau_px)

    def get(self, name, dtype):
        return vm3dgs_debug_get(self.h, name, dtype)

    def close(self):
        if self.h:
            vm3dgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ prefetch network
class Mlp:
    """The page-prefetch network of the library (vm3dgs_mlp_*): device
    memory of inputs, labels and outputs comes from torch tensors."""

    def __init__(self, dims, max_batch, stream=None):
        import torch
        if stream is None:
            # torch's current stream when it is a stream of its own; its default
            # stream has the handle 0, which the library reads as "a stream of
            # the network's own", so the calls below also order the two streams
            # on the host: torch's work before a call, the network's work before
            # the call returns (inputs may be torch temporaries)
            stream = torch.cuda.current_stream().cuda_stream
        self.dims = [int(d) for d in dims]
        arr = (C.c_uint32 * len(self.dims))(*self.dims)
        h = C.c_void_p()
        rc = lib().vm3dgs_mlp_create(arr, len(self.dims) - 1, int(max_batch), stream, C.byref(h))
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_mlp_create_error().decode())
        self.h = h
        self.n_params = int(lib().vm3dgs_mlp_n_params(h))

    def _check(self, rc):
        if rc != 0:
            raise Vm3dgsError(rc, lib().vm3dgs_mlp_last_error(self.h).decode())

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().vm3dgs_mlp_set_params(self.h, p.ctypes.data, p.size))

    def get_state(self):
        n = self.n_params
        p, m, v = np.zeros(n, np.float32), np.zeros(n, np.float32), np.zeros(n, np.float32)
        step = C.c_uint32()
        self._check(lib().vm3dgs_mlp_get_state(self.h, p.ctypes.data, m.ctypes.data, v.ctypes.data, n,
                                               C.byref(step)))
        return p, m, v, step.value

    def forward(self, x):
        import torch
        x = x.contiguous()
        z = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        torch.cuda.current_stream().synchronize()
        self._check(lib().vm3dgs_mlp_forward(self.h, x.data_ptr(), x.shape[0], z.data_ptr()))
        self.sync()
        return z

    def gradient(self, x, y):
        import torch
        x, y = x.contiguous(), y.contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = C.c_float()
        torch.cuda.current_stream().synchronize()
        self._check(lib().vm3dgs_mlp_gradient(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], g.data_ptr(),
                                              C.byref(loss)))
        self.sync()
        return g, loss.value

    def train_step(self, x, y, lr, want_loss=True):
        import torch
        loss = C.c_float()
        torch.cuda.current_stream().synchronize()
        self._check(lib().vm3dgs_mlp_train_step(self.h, x.data_ptr(), y.data_ptr(), x.shape[0], float(lr),
                                                C.byref(loss) if want_loss else None))
        self.sync()
        return loss.value if want_loss else None

    def save(self, path):
        self._check(lib().vm3dgs_mlp_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(lib().vm3dgs_mlp_load(self.h, str(path).encode()))

    def sync(self):
        self._check(lib().vm3dgs_mlp_sync(self.h))

    def close(self):
        if self.h:
            lib().vm3dgs_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
