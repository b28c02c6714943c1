"""Seeded synthetic scenes and camera trajectories.

This module only draws inputs: Gaussian attributes in the activated form the
paper stores after preprocessing (Sec. 3 "Scene Storage": decoded opacity and
scale, unit quaternion, no normals) and pinhole cameras.  It holds none of the
method's arithmetic, so both the HIP path and the CPU oracle consume it.

Scene arrays (all float32, C-contiguous):
    means   [n, 3]  metres, world z-up
    scales  [n, 3]  activated standard deviations (> 0)
    quats   [n, 4]  w, x, y, z (unit length)
    opacity [n]     in (0, 1)
    sh      [n, 16, 3] degree-3 SH coefficients, coefficient-major

Camera dict: view [4,4] (world -> camera, OpenCV axes: x right, y down,
z forward), cam_pos [3], fx, fy, cx, cy, znear.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Scene", "Camera", "look_at", "intrinsics", "scene_clusters", "orbit",
    "scene_terrain", "path_terrain", "scene_city", "path_city", "CONFIGS",
]


@dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    # axis-aligned extent used by trajectory generators (not by the method)
    bounds: tuple = None
    extra: dict = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means[idx].copy(), self.scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity[idx].copy(),
                     self.sh[idx].copy(), self.bounds, self.extra)


@dataclass
class Camera:
    view: np.ndarray      # [4, 4] float32 row-major
    cam_pos: np.ndarray   # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    znear: float = 0.2


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def intrinsics(width: int, height: int, fov_x_deg: float):
    """Horizontal field of view, square pixels, principal point at the centre."""
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return fx, fx, width / 2.0, height / 2.0


def look_at(eye, forward, width, height, fov_x_deg, znear=0.2, up=(0.0, 0.0, 1.0)):
    """Camera at ``eye`` looking along ``forward`` (world z-up)."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(forward, dtype=np.float64)
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    if np.linalg.norm(r) < 1e-9:          # looking straight up/down
        r = np.cross(f, np.array([0.0, 1.0, 0.0]))
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)                    # camera +y (down)
    R = np.stack([r, d, f])               # rows: camera axes in world
    T = -R @ eye
    V = np.eye(4)
    V[:3, :3] = R
    V[:3, 3] = T
    fx, fy, cx, cy = intrinsics(width, height, fov_x_deg)
    return Camera(_f32(V), _f32(eye), float(fx), float(fy), float(cx), float(cy), float(znear))


def _random_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _sh(rng, n, std=0.3, dc_offset=0.5, chunks=16):
    """SH coefficients N(0, std^2) (DC shifted by dc_offset), drawn in float32
    from `chunks` child streams of `rng` filled in parallel threads; the result
    depends only on the seed, not on the number of cores."""
    from concurrent.futures import ThreadPoolExecutor
    sh = np.empty((n, 16, 3), dtype=np.float32)
    flat = sh.reshape(-1)
    children = rng.spawn(chunks)
    bounds = np.linspace(0, flat.size, chunks + 1).astype(np.int64)

    def fill(i):
        children[i].standard_normal(out=flat[bounds[i]:bounds[i + 1]], dtype=np.float32)

    with ThreadPoolExecutor(max_workers=min(chunks, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(chunks)))
    sh *= np.float32(std)
    sh[:, 0, :] += np.float32(dc_offset)
    return sh


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _pack(means, scales, quats, opacity, sh, bounds=None, extra=None) -> Scene:
    return Scene(_f32(means), _f32(scales), _f32(quats), _f32(opacity), _f32(sh), bounds, extra)


# --------------------------------------------------------------------------
# Small parity scene: 8 isotropic clusters
# --------------------------------------------------------------------------
def scene_clusters(seed: int = 0, n_clusters: int = 8, per_cluster: int = 4096,
                   cluster_sigma: float = 2.0, cube: float = 10.0) -> Scene:
    """8 clusters (sigma 2 m) with centres uniform in a 20 m cube; 32,768 Gaussians.

    Draw order: centres, means, log-scales, quaternions, opacity, SH.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-cube, cube, size=(n_clusters, 3))
    means = (centres[:, None, :] + rng.normal(0.0, cluster_sigma, size=(n_clusters, per_cluster, 3))).reshape(-1, 3)
    n = means.shape[0]
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3)))
    quats = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    sh = _sh(rng, n)
    b = (means.min(0), means.max(0))
    return _pack(means, scales, quats, opacity, sh, bounds=b)


def scene_ties(seed: int = 0, copies: int = 4, per_cluster: int = 1024) -> Scene:
    """The cluster scene with every mean shared by ``copies`` consecutive
    Gaussians, whose other attributes are drawn for each: exact depth ties in
    every view (8 * per_cluster * copies Gaussians).

    Draw order: the cluster scene's (seed), then log-scales, quaternions,
    opacity and SH of all copies (seed + 1).
    """
    base = scene_clusters(seed, per_cluster=per_cluster)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    means = np.repeat(base.means, copies, axis=0)
    n = means.shape[0]
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3)))
    quats = _random_quats(rng, n)
    opacity = _sigmoid(rng.normal(0.0, 1.0, size=n))
    sh = _sh(rng, n)
    return _pack(means, scales, quats, opacity, sh, bounds=base.bounds)


def orbit(n_frames: int = 8, radius: float = 25.0, width: int = 320, height: int = 240,
          fov_x_deg: float = 60.0, height_z: float = 0.0):
    """Circle of ``radius`` in the z = 0 plane looking at the origin, angle 2 pi k / n."""
    cams = []
    for k in range(n_frames):
        a = 2.0 * math.pi * k / n_frames
        eye = np.array([radius * math.cos(a), radius * math.sin(a), height_z])
        cams.append(look_at(eye, -eye, width, height, fov_x_deg))
    return cams


# --------------------------------------------------------------------------
# Terrain + buildings (scene-scale configuration)
# --------------------------------------------------------------------------
def _terrain_params(rng, n_waves=8, amp_total=5.0, extent=100.0):
    amps = rng.uniform(0.2, 1.0, size=n_waves)
    amps *= amp_total / amps.sum()
    wl = rng.uniform(15.0, 120.0, size=n_waves)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=n_waves)
    k = np.stack([np.cos(ang), np.sin(ang)], 1) * (2.0 * math.pi / wl)[:, None]
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n_waves)
    return amps, k, ph


def _height(params, x, y):
    amps, k, ph = params
    h = np.zeros_like(x, dtype=np.float64)
    for a, kk, p in zip(amps, k, ph):
        h += a * np.sin(kk[0] * x + kk[1] * y + p)
    return h


def _height_grad(params, x, y):
    amps, k, ph = params
    gx = np.zeros_like(x, dtype=np.float64)
    gy = np.zeros_like(x, dtype=np.float64)
    for a, kk, p in zip(amps, k, ph):
        c = a * np.cos(kk[0] * x + kk[1] * y + p)
        gx += c * kk[0]
        gy += c * kk[1]
    return gx, gy


def _frame_quats(normals, rng):
    """Unit quaternions (w, x, y, z) whose local z axis is ``normals``, with a
    uniform random spin about it: the shortest rotation taking z to the normal,
    composed with a rotation about z."""
    n = normals / np.linalg.norm(normals, axis=1, keepdims=True)
    w1 = 1.0 + n[:, 2]
    x1 = -n[:, 1]
    y1 = n[:, 0].copy()
    flip = w1 < 1e-9                      # normal = -z: rotate by pi about x
    w1[flip], x1[flip], y1[flip] = 0.0, 1.0, 0.0
    nrm = np.sqrt(w1 * w1 + x1 * x1 + y1 * y1)
    w1 /= nrm; x1 /= nrm; y1 /= nrm
    th = rng.uniform(0.0, 2.0 * math.pi, size=n.shape[0])
    w2, z2 = np.cos(0.5 * th), np.sin(0.5 * th)
    return np.stack([w1 * w2, x1 * w2 + y1 * z2, y1 * w2 - x1 * z2, w1 * z2], 1)


def _mat_to_quat(R):
    """Rotation matrices [n,3,3] -> quaternions wxyz (w >= 0)."""
    m = R
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    q = np.zeros((m.shape[0], 4))
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr[c0] + 1.0, 1e-30)) * 2
    q[c0, 0] = 0.25 * s
    q[c0, 1] = (m[c0, 2, 1] - m[c0, 1, 2]) / s
    q[c0, 2] = (m[c0, 0, 2] - m[c0, 2, 0]) / s
    q[c0, 3] = (m[c0, 1, 0] - m[c0, 0, 1]) / s
    rest = ~c0
    i1 = rest & (m[:, 0, 0] > m[:, 1, 1]) & (m[:, 0, 0] > m[:, 2, 2])
    s = np.sqrt(np.maximum(1.0 + m[i1, 0, 0] - m[i1, 1, 1] - m[i1, 2, 2], 1e-30)) * 2
    q[i1, 0] = (m[i1, 2, 1] - m[i1, 1, 2]) / s
    q[i1, 1] = 0.25 * s
    q[i1, 2] = (m[i1, 0, 1] + m[i1, 1, 0]) / s
    q[i1, 3] = (m[i1, 0, 2] + m[i1, 2, 0]) / s
    i2 = rest & ~i1 & (m[:, 1, 1] > m[:, 2, 2])
    s = np.sqrt(np.maximum(1.0 + m[i2, 1, 1] - m[i2, 0, 0] - m[i2, 2, 2], 1e-30)) * 2
    q[i2, 0] = (m[i2, 0, 2] - m[i2, 2, 0]) / s
    q[i2, 1] = (m[i2, 0, 1] + m[i2, 1, 0]) / s
    q[i2, 2] = 0.25 * s
    q[i2, 3] = (m[i2, 1, 2] + m[i2, 2, 1]) / s
    i3 = rest & ~i1 & ~i2
    s = np.sqrt(np.maximum(1.0 + m[i3, 2, 2] - m[i3, 0, 0] - m[i3, 1, 1], 1e-30)) * 2
    q[i3, 0] = (m[i3, 1, 0] - m[i3, 0, 1]) / s
    q[i3, 1] = (m[i3, 0, 2] + m[i3, 2, 0]) / s
    q[i3, 2] = (m[i3, 1, 2] + m[i3, 2, 1]) / s
    q[i3, 3] = 0.25 * s
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    return q


def _catmull_rom_loop(ctrl, n_samples, step):
    """Closed Catmull-Rom spline through ``ctrl`` [k,2], resampled every ``step`` metres."""
    k = ctrl.shape[0]
    dense = []
    for i in range(k):
        p0, p1, p2, p3 = ctrl[(i - 1) % k], ctrl[i], ctrl[(i + 1) % k], ctrl[(i + 2) % k]
        t = np.linspace(0.0, 1.0, 400, endpoint=False)[:, None]
        dense.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t ** 2
                            + (-p0 + 3 * p1 - 3 * p2 + p3) * t ** 3))
    dense = np.concatenate(dense, 0)
    seg = np.linalg.norm(np.diff(np.concatenate([dense, dense[:1]], 0), axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    total = s[-1]
    want = (np.arange(n_samples) * step) % total
    x = np.interp(want, s, np.concatenate([dense[:, 0], dense[:1, 0]]))
    y = np.interp(want, s, np.concatenate([dense[:, 1], dense[:1, 1]]))
    return np.stack([x, y], 1), total


def _terrain_path_xy(seed, n_frames=300, step=1.0, n_ctrl=8):
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    r0 = n_frames * step / (2.0 * math.pi)
    ang = 2.0 * math.pi * np.arange(n_ctrl) / n_ctrl
    rad = r0 * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, size=n_ctrl))
    ctrl = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
    xy, total = _catmull_rom_loop(ctrl, n_frames, step)
    return xy


def scene_terrain(seed: int = 0, n_terrain: int = 3_000_000, n_building: int = 3_000_000,
                  n_buildings: int = 40, extent: float = 100.0, path_frames: int = 300) -> Scene:
    """200 x 200 m heightfield (8 sinusoids, amplitude <= 5 m) + 40 box buildings.

    Terrain Gaussians are flat and surface aligned (normal scale 0.02 m,
    in-plane about 0.7x the mean spacing); building Gaussians lie on the
    faces and roofs, the count per building drawn log-normal(0, 0.75).
    Building footprints keep 8 m clear of the camera path.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    params = _terrain_params(rng, extent=extent)
    # terrain
    x = rng.uniform(-extent, extent, size=n_terrain)
    y = rng.uniform(-extent, extent, size=n_terrain)
    z = _height(params, x, y)
    gx, gy = _height_grad(params, x, y)
    nrm = np.stack([-gx, -gy, np.ones_like(gx)], 1)
    spacing = math.sqrt((2 * extent) ** 2 / max(n_terrain, 1))
    t_means = np.stack([x, y, z], 1)
    t_scales = np.stack([0.7 * spacing * np.exp(rng.normal(0, 0.2, n_terrain)),
                         0.7 * spacing * np.exp(rng.normal(0, 0.2, n_terrain)),
                         np.full(n_terrain, 0.02)], 1)
    t_quats = _frame_quats(nrm, rng)
    # buildings, away from the camera path
    path = _terrain_path_xy(seed, path_frames)
    boxes = []
    tries = 0
    while len(boxes) < n_buildings and tries < 100000:
        tries += 1
        w, d = rng.uniform(10.0, 30.0, size=2)
        h = rng.uniform(10.0, 60.0)
        cx, cy = rng.uniform(-extent + 16, extent - 16, size=2)
        # distance from the path to the footprint rectangle
        dx = np.maximum(np.abs(path[:, 0] - cx) - w / 2, 0)
        dy = np.maximum(np.abs(path[:, 1] - cy) - d / 2, 0)
        if np.min(np.hypot(dx, dy)) < 8.0:
            continue
        if any(abs(cx - b[0]) < (w + b[2]) / 2 + 2 and abs(cy - b[1]) < (d + b[3]) / 2 + 2 for b in boxes):
            continue
        gxs = np.linspace(cx - w / 2, cx + w / 2, 9)
        gys = np.linspace(cy - d / 2, cy + d / 2, 9)
        GX, GY = np.meshgrid(gxs, gys)
        base = float(_height(params, GX, GY).min()) - 0.5
        boxes.append((cx, cy, w, d, h, base))
    weights = rng.lognormal(0.0, 0.75, size=len(boxes))
    counts = np.floor(weights / weights.sum() * n_building).astype(np.int64)
    counts[0] += n_building - counts.sum()
    bm, bs, bn = [], [], []
    for (cx, cy, w, d, h, base), c in zip(boxes, counts):
        areas = np.array([w * h, w * h, d * h, d * h, w * d])
        face = rng.choice(5, size=c, p=areas / areas.sum())
        u = rng.uniform(-0.5, 0.5, size=c)
        v = rng.uniform(0.0, 1.0, size=c)
        px = np.empty(c); py = np.empty(c); pz = np.empty(c); nn = np.zeros((c, 3))
        # faces: 0 = -y, 1 = +y, 2 = -x, 3 = +x, 4 = roof
        m = face == 0; px[m] = cx + u[m] * w; py[m] = cy - d / 2; pz[m] = base + v[m] * h; nn[m] = (0, -1, 0)
        m = face == 1; px[m] = cx + u[m] * w; py[m] = cy + d / 2; pz[m] = base + v[m] * h; nn[m] = (0, 1, 0)
        m = face == 2; px[m] = cx - w / 2; py[m] = cy + u[m] * d; pz[m] = base + v[m] * h; nn[m] = (-1, 0, 0)
        m = face == 3; px[m] = cx + w / 2; py[m] = cy + u[m] * d; pz[m] = base + v[m] * h; nn[m] = (1, 0, 0)
        m = face == 4; px[m] = cx + u[m] * w; py[m] = cy + (v[m] - 0.5) * d; pz[m] = base + h; nn[m] = (0, 0, 1)
        sp = math.sqrt(areas.sum() / max(c, 1))
        bm.append(np.stack([px, py, pz], 1))
        bs.append(np.stack([0.7 * sp * np.exp(rng.normal(0, 0.2, c)),
                            0.7 * sp * np.exp(rng.normal(0, 0.2, c)),
                            np.full(c, 0.02)], 1))
        bn.append(nn)
    b_means = np.concatenate(bm, 0) if bm else np.zeros((0, 3))
    b_scales = np.concatenate(bs, 0) if bs else np.zeros((0, 3))
    b_quats = _frame_quats(np.concatenate(bn, 0), rng) if bn else np.zeros((0, 4))
    means = np.concatenate([t_means, b_means], 0)
    scales = np.concatenate([t_scales, b_scales], 0)
    quats = np.concatenate([t_quats, b_quats], 0)
    n = means.shape[0]
    opacity = _sigmoid(rng.normal(2.0, 1.0, size=n))
    sh = _sh(rng, n)
    return _pack(means, scales, quats, opacity, sh,
                 bounds=(means.min(0), means.max(0)),
                 extra={"terrain": params, "boxes": boxes, "seed": seed})


def path_terrain(scene: Scene, n_frames: int = 300, width: int = 1920, height: int = 1080,
                 fov_x_deg: float = 70.0, eye_height: float = 1.7, step: float = 1.0):
    """Closed Catmull-Rom fly-through 1.7 m above the terrain, yaw along the motion."""
    seed = scene.extra["seed"]
    xy = _terrain_path_xy(seed, n_frames, step)
    params = scene.extra["terrain"]
    cams = []
    for i in range(n_frames):
        p = xy[i]
        q = xy[(i + 1) % n_frames]
        fwd = np.array([q[0] - p[0], q[1] - p[1], 0.0])
        if np.linalg.norm(fwd) < 1e-9:
            fwd = np.array([1.0, 0.0, 0.0])
        z = float(_height(params, np.array([p[0]]), np.array([p[1]]))[0]) + eye_height
        cams.append(look_at([p[0], p[1], z], fwd, width, height, fov_x_deg))
    return cams


# --------------------------------------------------------------------------
# City (LOD configuration), scalable so tests can run a small copy
# --------------------------------------------------------------------------
def scene_city(seed: int = 0, n: int = 50_000_000, size: float = 1000.0, block: float = 100.0,
               street: float = 20.0, color: str = "iid") -> Scene:
    """Street grid of 100 m blocks with 20 m streets; 1-6 buildings per block
    with log-normal heights clipped to 10-150 m; Gaussians split over ground,
    facades and roofs by area.

    color: "iid" draws every SH coefficient of every Gaussian independently
    (N(0, 0.3^2), DC + 0.5), as the cluster and terrain scenes do; "smooth"
    gives colours that vary smoothly over the surfaces (see _city_colours);
    "white" makes every Gaussian white with no view dependence, so that an
    image shows coverage (1 - final transmittance) alone."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = int(round(size / block))
    half = size / 2
    boxes = []
    for bi in range(nb):
        for bj in range(nb):
            x0 = -half + bi * block + street / 2
            y0 = -half + bj * block + street / 2
            inner = block - street
            k = int(rng.integers(1, 7))
            # split the block into a k-cell grid of lots
            gx = int(math.ceil(math.sqrt(k)))
            gy = int(math.ceil(k / gx))
            lw, ld = inner / gx, inner / gy
            for t in range(k):
                ix, iy = t % gx, t // gx
                w = lw * rng.uniform(0.55, 0.9)
                d = ld * rng.uniform(0.55, 0.9)
                cx = x0 + (ix + 0.5) * lw
                cy = y0 + (iy + 0.5) * ld
                h = float(np.clip(rng.lognormal(math.log(30.0), 0.6), 10.0, 150.0))
                boxes.append((cx, cy, w, d, h))
    ground_area = size * size
    face_areas = [2 * (w + d) * h + w * d for (_, _, w, d, h) in boxes]
    total_area = ground_area + sum(face_areas)
    n_ground = int(n * ground_area / total_area)
    per_box = np.floor(np.array(face_areas) / total_area * n).astype(np.int64)
    n_ground += n - n_ground - int(per_box.sum())
    # ground (flat z = 0)
    gx_ = rng.uniform(-half, half, size=n_ground)
    gy_ = rng.uniform(-half, half, size=n_ground)
    sp = math.sqrt(ground_area / max(n_ground, 1))
    parts_m = [np.stack([gx_, gy_, np.zeros(n_ground)], 1)]
    parts_s = [np.stack([0.7 * sp * np.exp(rng.normal(0, 0.2, n_ground)),
                         0.7 * sp * np.exp(rng.normal(0, 0.2, n_ground)),
                         np.full(n_ground, 0.02)], 1)]
    parts_n = [np.tile(np.array([[0.0, 0.0, 1.0]]), (n_ground, 1))]
    parts_o = [np.full(n_ground, -1, np.int32)]
    for b, ((cx, cy, w, d, h), c) in enumerate(zip(boxes, per_box)):
        if c <= 0:
            continue
        areas = np.array([w * h, w * h, d * h, d * h, w * d])
        face = rng.choice(5, size=c, p=areas / areas.sum())
        u = rng.uniform(-0.5, 0.5, size=c)
        v = rng.uniform(0.0, 1.0, size=c)
        px = np.empty(c); py = np.empty(c); pz = np.empty(c); nn = np.zeros((c, 3))
        m = face == 0; px[m] = cx + u[m] * w; py[m] = cy - d / 2; pz[m] = v[m] * h; nn[m] = (0, -1, 0)
        m = face == 1; px[m] = cx + u[m] * w; py[m] = cy + d / 2; pz[m] = v[m] * h; nn[m] = (0, 1, 0)
        m = face == 2; px[m] = cx - w / 2; py[m] = cy + u[m] * d; pz[m] = v[m] * h; nn[m] = (-1, 0, 0)
        m = face == 3; px[m] = cx + w / 2; py[m] = cy + u[m] * d; pz[m] = v[m] * h; nn[m] = (1, 0, 0)
        m = face == 4; px[m] = cx + u[m] * w; py[m] = cy + (v[m] - 0.5) * d; pz[m] = h; nn[m] = (0, 0, 1)
        spb = math.sqrt(areas.sum() / c)
        parts_m.append(np.stack([px, py, pz], 1))
        parts_s.append(np.stack([0.7 * spb * np.exp(rng.normal(0, 0.2, c)),
                                 0.7 * spb * np.exp(rng.normal(0, 0.2, c)),
                                 np.full(c, 0.02)], 1))
        parts_n.append(nn)
        parts_o.append(np.full(c, b, np.int32))
    means = np.concatenate(parts_m, 0)
    scales = np.concatenate(parts_s, 0)
    quats = _frame_quats(np.concatenate(parts_n, 0), rng)
    nn_ = means.shape[0]
    opacity = _sigmoid(rng.normal(2.0, 1.0, size=nn_))
    if color == "iid":
        sh = _sh(rng, nn_)
    elif color == "smooth":
        sh = _city_colours(rng, means, np.concatenate(parts_o, 0), boxes, size, block, street)
    elif color == "white":
        sh = np.zeros((nn_, 16, 3), np.float32)
        sh[:, 0, :] = np.float32(0.5 / SH_C0)
    else:
        raise ValueError(f"unknown city colour model {color!r}")
    return _pack(means, scales, quats, opacity, sh, bounds=(means.min(0), means.max(0)),
                 extra={"boxes": boxes, "size": size, "block": block, "street": street, "seed": seed,
                        "color": color})


# degree-0 real SH constant 1 / (2 sqrt(pi)): colour = SH_C0 * DC + 0.5 + higher degrees
SH_C0 = 0.28209479177387814


def _waves(rng, d, n_waves, wl_min, wl_max):
    """n_waves plane waves in d dimensions: random unit directions,
    wavelengths log-uniform in [wl_min, wl_max], random phases."""
    k = rng.normal(size=(n_waves, d))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    wl = np.exp(rng.uniform(math.log(wl_min), math.log(wl_max), size=n_waves))
    return k * (2 * math.pi / wl)[:, None], rng.uniform(0, 2 * math.pi, size=n_waves)


def _field(pts, waves, sd):
    """Sum of the plane waves at pts, scaled to standard deviation sd."""
    k, ph = waves
    v = np.zeros(pts.shape[0])
    for i in range(len(ph)):
        arg = np.full(pts.shape[0], ph[i])
        for j in range(pts.shape[1]):
            arg += pts[:, j] * k[i, j]
        v += np.sin(arg)
    return (v * (sd * math.sqrt(2.0 / len(ph)))).astype(np.float32)


def _city_colours(rng, means, owner, boxes, size, block, street, chunk=1_000_000):
    """Spatially smooth colours for the city, as a captured scene's colours
    are correlated over its surfaces.  Albedo (rgb in [0, 1]):
      ground   asphalt grey 0.30 on the streets, 0.50 on the blocks, each
               channel plus a field of 6 plane waves (wavelengths 6-60 m,
               standard deviation 0.06);
      building a base colour per building, U[0.30, 0.75] per channel, plus a
               3-D field of 6 plane waves (wavelengths 4-30 m, sd 0.05).
    DC = (albedo - 0.5) / SH_C0 + N(0, 0.01^2) per Gaussian (fine grain).
    Degrees 1-3: one set of 15 x 3 coefficients N(0, 0.04^2) for the ground
    and one per building (shared view dependence, so a surface keeps one
    sheen), plus N(0, 0.004^2) per Gaussian."""
    n = means.shape[0]
    nb = len(boxes)
    base = rng.uniform(0.30, 0.75, size=(nb, 3)).astype(np.float32)
    hi_ground = rng.normal(0.0, 0.04, size=(15, 3)).astype(np.float32)
    hi_build = rng.normal(0.0, 0.04, size=(nb, 15, 3)).astype(np.float32)
    g_waves = [_waves(rng, 2, 6, 6.0, 60.0) for _ in range(3)]
    b_waves = [_waves(rng, 3, 6, 4.0, 30.0) for _ in range(3)]
    noise_rng = np.random.Generator(np.random.PCG64(int(rng.integers(1 << 62))))
    hi_all = np.concatenate([hi_build, hi_ground[None]], 0)   # owner -1 (ground) reads the last row
    sh = _sh(noise_rng, n, std=1.0, dc_offset=0.0)
    hi_flat = hi_all.reshape(nb + 1, 45)

    def fill(s0):
        s1 = min(n, s0 + chunk)
        m = means[s0:s1]
        own = owner[s0:s1]
        alb = np.empty((s1 - s0, 3), np.float32)
        g = own < 0
        if g.any():
            xy = m[g, :2]
            # streets are centred on x = -size/2 + k * block (likewise y)
            fx = np.mod(xy[:, 0] + 0.5 * size, block)
            fy = np.mod(xy[:, 1] + 0.5 * size, block)
            on_street = (np.minimum(fx, block - fx) < street / 2) | (np.minimum(fy, block - fy) < street / 2)
            lvl = np.where(on_street, 0.30, 0.50).astype(np.float32)
            for c in range(3):
                alb[g, c] = lvl + _field(xy, g_waves[c], 0.06)
        b = ~g
        if b.any():
            for c in range(3):
                alb[b, c] = base[own[b], c] + _field(m[b], b_waves[c], 0.05)
        np.clip(alb, 0.02, 0.98, out=alb)
        blk = sh[s0:s1]
        blk[:, 0, :] *= np.float32(0.01)
        blk[:, 0, :] += (alb - np.float32(0.5)) / np.float32(SH_C0)
        blk[:, 1:, :] *= np.float32(0.004)
        blk[:, 1:, :] += np.take(hi_flat, own, axis=0, mode="wrap").reshape(s1 - s0, 15, 3)

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(fill, range(0, n, chunk)))
    return sh


def path_city(scene: Scene, n_frames: int = 600, width: int = 1920, height: int = 1080,
              fov_x_deg: float = 70.0, seed: int = None):
    """Street level (1.7 m) for the first third, ascending to 150 m in the
    second, aerial at 150 m pitched down 35 degrees in the last third."""
    ex = scene.extra
    size, block = ex["size"], ex["block"]
    rng = np.random.Generator(np.random.PCG64(ex["seed"] + 104729 if seed is None else seed))
    half = size / 2
    n_st = int(round(size / block))
    # streets run along x = -half + k*block (k = 0..n), same for y
    third = max(n_frames // 3, 1)
    # street segment: along one street line, 1 m/frame scaled to the scene size
    k = int(rng.integers(1, n_st))
    line = -half + k * block
    step = min(1.0, (size * 0.8) / max(third, 1))
    x0 = -half * 0.8
    cams = []
    heading = 0.0
    for i in range(n_frames):
        if i < third:
            x = x0 + i * step
            pos = np.array([x, line, 1.7]); fwd = np.array([1.0, 0.0, 0.0])
        elif i < 2 * third:
            t = (i - third) / max(third, 1)
            x = x0 + third * step + (i - third) * step * 0.5
            pos = np.array([x, line, 1.7 + t * (150.0 - 1.7)])
            pitch = -math.radians(35.0) * t
            fwd = np.array([math.cos(pitch), 0.0, math.sin(pitch)])
        else:
            t = (i - 2 * third) / max(n_frames - 2 * third, 1)
            heading = 2.0 * math.pi * t
            r = half * 0.5
            pos = np.array([r * math.cos(heading), r * math.sin(heading), 150.0])
            tang = np.array([-math.sin(heading), math.cos(heading), 0.0])
            pitch = -math.radians(35.0)
            fwd = np.array([tang[0] * math.cos(pitch), tang[1] * math.cos(pitch), math.sin(pitch)])
        cams.append(look_at(pos, fwd, width, height, fov_x_deg))
    return cams


# Per-configuration parameters of the VM path (page size, pool, buffers, ...).
CONFIGS = {
    "clusters32k": dict(page_size=256, pool_pages=64, lod_levels=1, img=(320, 240),
                        idbuf=(80, 60), fov=60.0, cell=0.5, frames=8),
    "terrain6m": dict(page_size=1024, pool_pages=1465, lod_levels=1, img=(1920, 1080),
                      idbuf=(240, 135), fov=70.0, cell=1.0, frames=300),
    "city50m_lod": dict(page_size=1024, pool_pages=3907, lod_levels=3, img=(1920, 1080),
                        idbuf=(240, 135), fov=70.0, cell=2.0, frames=600),
}
