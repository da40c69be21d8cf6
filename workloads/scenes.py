"""Seeded synthetic scenes, sensor poses and range images.

This module only *generates inputs*: analytic box scenes, camera poses, and
range images cast analytically against those boxes (plus sensor noise,
dropouts and dead pixels).  It holds none of the pose-scoring method's
arithmetic -- no meshification, no rasterization, no cost table, no SE(3)
Jacobians -- so that the FP64 oracle and the GPU library can both consume
its output without sharing code with each other.

Conventions (also those of the library):
  * camera axes follow OpenCV: x right, y down, z forward;
  * a pose ``T_wc`` is a 3x4 float64 matrix [R | t] mapping camera
    coordinates to world coordinates (the sensor pose in the map frame);
  * range images hold z-depth (distance along the optical axis, metres);
    0 encodes "no return", NaN a dead pixel;
  * the world frame has z pointing up.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation


@dataclass(frozen=True)
class Camera:
    """Pinhole intrinsics.  Pixel (u, v) has its centre at integer (u, v)."""
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.1
    z_far: float = 16.0

    def astuple(self):
        return (self.fx, self.fy, self.cx, self.cy, self.width, self.height,
                self.z_near, self.z_far)


KINECT = Camera(525.0, 525.0, 319.5, 239.5, 640, 480)
TINY = Camera(52.5, 52.5, 31.5, 23.5, 64, 48)
QVGA = Camera(262.5, 262.5, 159.5, 119.5, 320, 240)
WIDE = Camera(640.0, 640.0, 639.5, 479.5, 1280, 960)


@dataclass
class Door:
    """A rectangular opening in one wall of the room.  Rays that leave the
    room through it hit nothing (the sensor reports no return)."""
    axis: int          # wall normal axis (0 = x, 1 = y)
    side: int          # 0 = the wall at room_lo[axis], 1 = the wall at room_hi[axis]
    lo: tuple          # (a_lo, z_lo) along the other horizontal axis and z
    hi: tuple


@dataclass
class Scene:
    """Camera-inside room (an axis-aligned box seen from inside) plus solid
    axis-aligned boxes, optionally with door openings."""
    room_lo: np.ndarray
    room_hi: np.ndarray
    boxes: np.ndarray                        # [K, 2, 3] (lo, hi)
    doors: list = field(default_factory=list)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

def random_box_room(seed: int, size=(4.0, 4.0, 2.5), n_boxes=8,
                    side=(0.2, 0.8), margin=0.3, doors=()) -> Scene:
    """Room [0,sx]x[0,sy]x[0,sz] with ``n_boxes`` boxes standing on the floor,
    sides drawn from U[side].  Box corners are rounded to 1/64 m so that
    they are exact in float32."""
    rng = np.random.default_rng(seed)
    sx, sy, sz = size
    boxes = []
    for _ in range(n_boxes):
        w, d, h = rng.uniform(side[0], side[1], size=3)
        x0 = rng.uniform(margin, sx - margin - w)
        y0 = rng.uniform(margin, sy - margin - d)
        lo = np.array([x0, y0, 0.0])
        hi = np.array([x0 + w, y0 + d, h])
        boxes.append(np.stack([np.round(lo * 64) / 64, np.round(hi * 64) / 64]))
    return Scene(np.zeros(3), np.array(size, dtype=np.float64),
                 np.array(boxes, dtype=np.float64).reshape(-1, 2, 3), list(doors))


def corridor_scene(seed: int, length=60.0, width=2.5, height=2.7,
                   n_boxes=60, side=(0.2, 0.8)) -> Scene:
    """Long corridor along +x with clutter boxes along both walls."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(n_boxes):
        w, d, h = rng.uniform(side[0], side[1], size=3)
        x0 = rng.uniform(0.5, length - 0.5 - w)
        y0 = 0.05 if rng.random() < 0.5 else width - 0.05 - d
        lo = np.array([x0, y0, 0.0])
        hi = np.array([x0 + w, y0 + d, h])
        boxes.append(np.stack([np.round(lo * 64) / 64, np.round(hi * 64) / 64]))
    return Scene(np.zeros(3), np.array([length, width, height]),
                 np.array(boxes).reshape(-1, 2, 3), [])


# --------------------------------------------------------------------------
# poses
# --------------------------------------------------------------------------

def look_pose(position, yaw, pitch=0.0, roll=0.0) -> np.ndarray:
    """T_wc for a camera at ``position`` whose optical axis has the given yaw
    (about world z, from +x) and pitch (positive = up); roll about the axis."""
    f = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f], axis=1)
    if roll:
        R = R @ Rotation.from_rotvec(np.array([0.0, 0.0, roll])).as_matrix()
    T = np.zeros((3, 4))
    T[:, :3] = R
    T[:, 3] = position
    return T


def perturb(T: np.ndarray, rng, trans, rot_rad, fixed=False) -> np.ndarray:
    """Offset a pose by a translation and a rotation.

    fixed=True : exactly ``trans`` metres in a uniformly random direction and
                 exactly ``rot_rad`` about a uniformly random axis;
    fixed=False: per-axis N(0, trans) and rotation vector N(0, rot_rad).
    The rotation is applied in the camera frame (right composition)."""
    if fixed:
        d = rng.normal(size=3); d *= trans / np.linalg.norm(d)
        a = rng.normal(size=3); a *= rot_rad / np.linalg.norm(a)
    else:
        d = rng.normal(scale=trans, size=3)
        a = rng.normal(scale=rot_rad, size=3)
    out = T.copy()
    out[:, :3] = T[:, :3] @ Rotation.from_rotvec(a).as_matrix()
    out[:, 3] = T[:, 3] + d
    return out


def circle_views(seed: int, center, n: int, radius=1.0, height=(1.2, 1.6),
                 yaw_jitter=np.deg2rad(20), pitch=np.deg2rad(15)):
    """``n`` outward-looking poses on a horizontal circle around ``center``."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        ang = 2 * np.pi * k / n + rng.uniform(-0.1, 0.1)
        pos = np.array([center[0] + radius * np.cos(ang), center[1] + radius * np.sin(ang),
                        rng.uniform(*height)])
        out.append(look_pose(pos, ang + rng.uniform(-yaw_jitter, yaw_jitter),
                             rng.uniform(-pitch, pitch)))
    return out


def inward_views(seed: int, scene: Scene, n: int, frac=0.75, height=(1.2, 1.7),
                 pitch_deg=(-35.0, -10.0), aim_jitter=0.6, phase=0.0):
    """``n`` poses spread over an ellipse at ``frac`` of the room's half
    extents, each looking across the room at a point within ``aim_jitter`` m
    of its centre, tilted down by a pitch drawn from ``pitch_deg``: every view
    sees floor, far walls and boxes (no single plane fills the frame)."""
    rng = np.random.default_rng(seed)
    c = 0.5 * (scene.room_lo + scene.room_hi)
    half = 0.5 * (scene.room_hi - scene.room_lo)
    out = []
    for k in range(n):
        ang = 2 * np.pi * (k + phase) / n + rng.uniform(-0.1, 0.1)
        pos = np.array([c[0] + frac * half[0] * np.cos(ang), c[1] + frac * half[1] * np.sin(ang),
                        rng.uniform(*height)])
        tgt = c[:2] + rng.uniform(-aim_jitter, aim_jitter, 2)
        yaw = np.arctan2(tgt[1] - pos[1], tgt[0] - pos[0])
        out.append(look_pose(pos, yaw, np.deg2rad(rng.uniform(*pitch_deg))))
    return out


# --------------------------------------------------------------------------
# analytic range images
# --------------------------------------------------------------------------

def _rays(cam: Camera, T: np.ndarray):
    u = np.arange(cam.width, dtype=np.float64)
    v = np.arange(cam.height, dtype=np.float64)
    uu, vv = np.meshgrid(u, v)
    rc = np.stack([(uu - cam.cx) / cam.fx, (vv - cam.cy) / cam.fy, np.ones_like(uu)], -1)
    rw = rc @ T[:, :3].T          # world direction; parameter along it == z-depth
    return rw, T[:, 3]


def analytic_depth(scene: Scene, cam: Camera, T: np.ndarray, z_cut=np.inf) -> np.ndarray:
    """Exact (FP64) z-depth of the first surface hit for every pixel; +inf
    where the ray leaves through a door opening.  Boxes entirely behind the
    camera or entirely beyond depth ``z_cut`` are skipped: their hits could
    only lie beyond z_cut (callers treat such depths alike)."""
    rw, o = _rays(cam, T)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / rw
        # leaving the room interior
        t_hi = (scene.room_hi - o) * inv
        t_lo = (scene.room_lo - o) * inv
        t_exit_ax = np.where(rw > 0, t_hi, np.where(rw < 0, t_lo, np.inf))
        ax = np.argmin(t_exit_ax, axis=-1)
        t_exit = np.take_along_axis(t_exit_ax, ax[..., None], -1)[..., 0]
        depth = t_exit.copy()
        if scene.doors:
            p = o + rw * t_exit[..., None]
            for d in scene.doors:
                other = 1 - d.axis
                on_wall = (ax == d.axis) & ((rw[..., d.axis] > 0) == (d.side == 1))
                inside = ((p[..., other] >= d.lo[0]) & (p[..., other] <= d.hi[0]) &
                          (p[..., 2] >= d.lo[1]) & (p[..., 2] <= d.hi[1]))
                depth = np.where(on_wall & inside, np.inf, depth)
        H, W = depth.shape
        for lo, hi in scene.boxes:
            corners = np.array([[lo[0] if i & 1 else hi[0], lo[1] if i & 2 else hi[1], lo[2] if i & 4 else hi[2]]
                                for i in range(8)])
            cc = (corners - o) @ T[:, :3]                  # camera-frame corners
            zc = cc[:, 2]
            if zc.max() <= 0.0 or zc.min() > z_cut:
                continue
            # pixels whose ray can meet the box: with every corner in front
            # of the camera, inside the rectangle of the projected corners
            # (one pixel of margin); otherwise the whole image
            r0, r1, c0, c1 = 0, H, 0, W
            if zc.min() > 1e-9:
                u = cam.fx * cc[:, 0] / zc + cam.cx
                v = cam.fy * cc[:, 1] / zc + cam.cy
                c0, c1 = max(0, int(np.floor(u.min())) - 1), min(W, int(np.ceil(u.max())) + 2)
                r0, r1 = max(0, int(np.floor(v.min())) - 1), min(H, int(np.ceil(v.max())) + 2)
                if c0 >= c1 or r0 >= r1:
                    continue
            sub = (slice(r0, r1), slice(c0, c1))
            t1 = (lo - o) * inv[sub]
            t2 = (hi - o) * inv[sub]
            tn = np.nanmax(np.minimum(t1, t2), axis=-1)
            tf = np.nanmin(np.maximum(t1, t2), axis=-1)
            hit = (tn <= tf) & (tn > 0)
            d = depth[sub]
            depth[sub] = np.where(hit & (tn < d), tn, d)
    return depth


def range_image(scene: Scene, cam: Camera, T: np.ndarray, seed: int, noise_rel=0.01,
                z_max=8.0, dropout=0.0, dead=0.0) -> np.ndarray:
    """Simulated depth sensor: analytic depth, multiplicative N(0, noise_rel)
    noise, returns beyond ``z_max`` reported as 0 (no return), a fraction
    ``dropout`` of pixels forced to no return and a fraction ``dead`` to NaN.
    Returns float32 [H, W]."""
    rng = np.random.default_rng(seed)
    z = analytic_depth(scene, cam, T, z_cut=z_max)
    if noise_rel:
        z = z * (1.0 + noise_rel * rng.standard_normal(z.shape))
    z = np.where(np.isfinite(z) & (z <= z_max), z, 0.0)
    if dropout:
        z = np.where(rng.random(z.shape) < dropout, 0.0, z)
    if dead:
        z = np.where(rng.random(z.shape) < dead, np.nan, z)
    return z.astype(np.float32)


# --------------------------------------------------------------------------
# surface intensity (inputs of the color term): a smooth procedural albedo,
# intensity images of the scene and per-triangle intensities of a mesh
# --------------------------------------------------------------------------

def albedo(points) -> np.ndarray:
    """Intensity in [0.05, 0.95] of world points: 0.5 plus 0.15 times the sum
    of three sinusoids along the world axes (wavelengths 0.7, 0.9, 0.8 m),
    so that every axis-aligned surface shows a pattern."""
    p = np.asarray(points, np.float64)
    return 0.5 + 0.15 * (np.sin(2 * np.pi * p[..., 0] / 0.7) + np.sin(2 * np.pi * p[..., 1] / 0.9)
                         + np.sin(2 * np.pi * p[..., 2] / 0.8))


def intensity_image(scene: Scene, cam: Camera, T: np.ndarray, seed: int, noise=0.01, z_max=8.0) -> np.ndarray:
    """Intensity a co-registered camera reports: the albedo of the first
    surface each pixel sees plus N(0, noise); NaN where the ray leaves the
    room or its hit lies beyond ``z_max``.  Float32 [H, W]."""
    rng = np.random.default_rng(seed)
    rw, o = _rays(cam, T)
    z = analytic_depth(scene, cam, T, z_cut=z_max)
    ok = np.isfinite(z) & (z <= z_max)
    p = o + rw * np.where(ok, z, 0.0)[..., None]
    val = albedo(p) + noise * rng.standard_normal(z.shape)
    return np.where(ok, val, np.nan).astype(np.float32)


def triangle_albedo(xyz, tri) -> np.ndarray:
    """Albedo at each triangle's centroid, float32 [T] (NaN for triangles
    with a non-finite vertex)."""
    xyz = np.asarray(xyz, np.float64)
    tri = np.asarray(tri, np.int64)
    if len(tri) == 0:
        return np.zeros(0, np.float32)
    with np.errstate(invalid="ignore"):
        c = xyz[tri].mean(axis=1)
        return albedo(c).astype(np.float32)


# --------------------------------------------------------------------------
# procedural triangulation of the analytic scene (map meshes of the tiny and
# corridor workloads, and closed-form test geometry)
# --------------------------------------------------------------------------

def _grid_rect(origin, e1, e2, n1, n2, flip=False):
    """Vertices and triangles of a planar rectangle origin + a*e1 + b*e2,
    a, b in [0, 1], split into n1 x n2 quads (two triangles each)."""
    a = np.linspace(0.0, 1.0, n1 + 1)
    b = np.linspace(0.0, 1.0, n2 + 1)
    aa, bb = np.meshgrid(a, b, indexing="ij")
    xyz = origin + aa[..., None] * e1 + bb[..., None] * e2
    idx = np.arange((n1 + 1) * (n2 + 1)).reshape(n1 + 1, n2 + 1)
    q00 = idx[:-1, :-1].ravel(); q01 = idx[:-1, 1:].ravel()
    q10 = idx[1:, :-1].ravel(); q11 = idx[1:, 1:].ravel()
    if flip:
        tri = np.concatenate([np.stack([q00, q11, q01], 1), np.stack([q00, q10, q11], 1)])
    else:
        tri = np.concatenate([np.stack([q00, q01, q11], 1), np.stack([q00, q11, q10], 1)])
    # interleave the two triangles of each quad so that consecutive ids are neighbours
    nq = q00.size
    order = np.stack([np.arange(nq), np.arange(nq) + nq], 1).ravel()
    return xyz.reshape(-1, 3), tri[order]


def triangulate_scene(scene: Scene, cell=0.25, box_cells=1):
    """Triangle mesh of the room surfaces (on a ``cell`` grid) and of every box
    (``box_cells`` x ``box_cells`` quads per face).  All triangles are class
    0 (free-occupied).  Returns (xyz f32 [V,3], tri i32 [T,3], cls u8 [T])."""
    parts = []
    lo, hi = scene.room_lo, scene.room_hi
    ext = hi - lo
    n = np.maximum(1, np.round(ext / cell).astype(int))
    E = np.eye(3)
    for axis in range(3):
        a1, a2 = [k for k in range(3) if k != axis]
        for side in (0, 1):
            o = lo.copy(); o[axis] = hi[axis] if side else lo[axis]
            parts.append(_grid_rect(o, E[a1] * ext[a1], E[a2] * ext[a2], n[a1], n[a2], flip=bool(side)))
    for blo, bhi in scene.boxes:
        bext = bhi - blo
        for axis in range(3):
            a1, a2 = [k for k in range(3) if k != axis]
            for side in (0, 1):
                o = blo.copy(); o[axis] = bhi[axis] if side else blo[axis]
                parts.append(_grid_rect(o, E[a1] * bext[a1], E[a2] * bext[a2], box_cells, box_cells,
                                        flip=bool(side)))
    xyz, tri, off = [], [], 0
    for v, t in parts:
        xyz.append(v); tri.append(t + off); off += len(v)
    xyz = np.concatenate(xyz).astype(np.float32)
    tri = np.concatenate(tri).astype(np.int32)
    return xyz, tri, np.zeros(len(tri), np.uint8)


def plane_mesh(n_per_side=8, extent=4.0, z0=2.0, slope=(0.25, 0.125)):
    """A tilted plane z = z0 + sx*x + sy*y over [-extent, extent]^2 on a
    dyadic grid, so that every vertex is exact in float32."""
    k = np.linspace(-extent, extent, n_per_side + 1)
    xx, yy = np.meshgrid(k, k, indexing="ij")
    zz = z0 + slope[0] * xx + slope[1] * yy
    xyz = np.stack([xx, yy, zz], -1).reshape(-1, 3)
    idx = np.arange(xyz.shape[0]).reshape(n_per_side + 1, n_per_side + 1)
    q00 = idx[:-1, :-1].ravel(); q01 = idx[:-1, 1:].ravel()
    q10 = idx[1:, :-1].ravel(); q11 = idx[1:, 1:].ravel()
    tri = np.concatenate([np.stack([q00, q01, q11], 1), np.stack([q00, q11, q10], 1)])
    return xyz.astype(np.float32), tri.astype(np.int32), np.zeros(len(tri), np.uint8)


def concat_meshes(meshes):
    """Union of meshes (xyz, tri, cls) with vertex-index offsets."""
    xyz, tri, cls, off = [], [], [], 0
    for v, t, c in meshes:
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
    return (np.concatenate(xyz).astype(np.float32), np.concatenate(tri).astype(np.int32),
            np.concatenate(cls).astype(np.uint8))
