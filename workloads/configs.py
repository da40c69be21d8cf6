"""The five seeded synthetic workloads of the pose-scoring path.

The paper evaluates on an RGB-D office sequence (its Section VI), which is not
available here; these synthetic scenes stand in for it with the same sensor
shape (Kinect-like 640x480 z-depth), indoor room scale, and the inter-scan
displacement the paper reports (about 0.15 m).  Every array is seeded.

A workload whose map is the union of meshified range images (kinect,
differentiation) carries the *range images and meshing parameters*; the
consumer meshifies them (the oracle in tests, the GPU library in the bench),
because meshification is part of the method and does not live here.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import scenes as S


@dataclass
class Workload:
    name: str
    cam: S.Camera
    scene: S.Scene
    T_true: np.ndarray                 # [3,4] ground-truth pose of the query scan
    scan_depth: np.ndarray             # [H,W] f32 range image of the query scan
    poses: np.ndarray                  # [B,3,4] candidate poses
    z_min: float = 0.5
    z_max: float = 8.0
    eps: float = 0.1
    map_mesh: tuple | None = None      # (xyz, tri, cls) when the map is procedural
    views: list = field(default_factory=list)        # [T_wc] of meshified map views
    view_depths: list = field(default_factory=list)  # [H,W] f32 range images
    stride: int = 1
    max_edge: float = 0.1
    smooth_radius: int = 0             # node smoothing window half-width of the map meshing
    map_color: np.ndarray | None = None    # [T] f32 triangle intensities of map_mesh (color term)
    scan_color: np.ndarray | None = None   # [H,W] f32 intensity image of the query scan


def _room_center(scene):
    return 0.5 * (scene.room_lo + scene.room_hi)


def tiny(seed: int = 0) -> Workload:
    """64x48 camera in a 4x4x2.5 m room with 8 boxes, procedural mesh of
    2,304 wall triangles (0.25 m grid) + 96 box triangles; one candidate
    pose 5 cm / 2 degrees from the truth."""
    rng = np.random.default_rng(seed)
    scene = S.random_box_room(seed, (4.0, 4.0, 2.5), 8)
    mesh = S.triangulate_scene(scene, cell=0.25)
    c = _room_center(scene)
    T = S.look_pose(np.array([c[0], c[1], 1.2]), rng.uniform(0, 2 * np.pi), 0.0)
    depth = S.range_image(scene, S.TINY, T, seed + 100, noise_rel=0.01)
    cand = S.perturb(T, rng, 0.05, np.deg2rad(2.0), fixed=True)
    return Workload("tiny", S.TINY, scene, T, depth, cand[None], map_mesh=mesh)


def _meshified_room(seed, n_views, stride, cam, dropout=0.02, size=(6.0, 5.0, 2.8), n_boxes=16):
    door = S.Door(axis=0, side=1, lo=(1.5, 0.0), hi=(2.5, 2.1))
    scene = S.random_box_room(seed, size, n_boxes, doors=[door])
    views = S.inward_views(seed + 7, scene, n_views)
    depths = [S.range_image(scene, cam, T, seed * 1000 + k, noise_rel=0.01, dropout=dropout)
              for k, T in enumerate(views)]
    return scene, views, depths


def _held_out_pose(scene, seed):
    """A query pose of the same family as the map views, at an angle none of
    them takes."""
    T = S.inward_views(seed, scene, 1, phase=0.37)[0]
    return T, np.random.default_rng(seed)


def kinect(seed: int = 1, n_poses: int = 64) -> Workload:
    """640x480 Kinect-like camera; map = 20 meshified views at stride 8 with
    node smoothing radius 4 (186,440 triangles, free-occupied plus
    free-unknown); 64 candidates drawn N(0, 3 cm) / N(0, 1.5 deg) per axis
    around the held-out truth."""
    cam = S.KINECT
    scene, views, depths = _meshified_room(seed, 20, 8, cam)
    T, rng = _held_out_pose(scene, seed + 11)
    depth = S.range_image(scene, cam, T, seed + 13, noise_rel=0.01, dropout=0.02)
    poses = np.stack([S.perturb(T, rng, 0.03, np.deg2rad(1.5)) for _ in range(n_poses)])
    return Workload("kinect", cam, scene, T, depth, poses, views=views, view_depths=depths,
                    stride=8, max_edge=0.1 * 8 / 2, smooth_radius=4)


def differentiation(seed: int = 1, n_poses: int = 64) -> Workload:
    """640x480; map = 27 meshified views at stride 4 with node smoothing
    radius 4 (27 x 37,842 = 1,021,734 triangles); 64 candidates exactly
    10 cm / 5 deg from the truth."""
    cam = S.KINECT
    scene, views, depths = _meshified_room(seed, 27, 4, cam)
    T, rng = _held_out_pose(scene, seed + 11)
    depth = S.range_image(scene, cam, T, seed + 13, noise_rel=0.01, dropout=0.02)
    poses = np.stack([S.perturb(T, rng, 0.10, np.deg2rad(5.0), fixed=True) for _ in range(n_poses)])
    return Workload("differentiation", cam, scene, T, depth, poses, views=views,
                    view_depths=depths, stride=4, max_edge=0.1 * 4 / 2, smooth_radius=4)


def wide(seed: int = 4, n_poses: int = 256, cell=0.018) -> Workload:
    """1280x960 camera in a 60 m corridor with clutter, procedural mesh on a
    ~1.8 cm grid (about 4M triangles); 10% dead pixels; 256 candidates."""
    cam = S.WIDE
    scene = S.corridor_scene(seed)
    mesh = S.triangulate_scene(scene, cell=cell, box_cells=8)
    rng = np.random.default_rng(seed)
    T = S.look_pose(np.array([5.0, 1.25, 1.4]), 0.0 + rng.uniform(-0.2, 0.2), rng.uniform(-0.1, 0.1))
    depth = S.range_image(scene, cam, T, seed + 13, noise_rel=0.01, dead=0.10)
    poses = np.stack([S.perturb(T, rng, 0.03, np.deg2rad(1.5)) for _ in range(n_poses)])
    return Workload("wide", cam, scene, T, depth, poses, map_mesh=mesh)



def textured_wall(seed: int = 8, n_poses: int = 8, cell=0.02) -> Workload:
    """A QVGA camera 1.5 m in front of a wall that fills its view (empty
    4x4x2.5 m room, procedural mesh on a 2 cm grid, ~0.36M triangles) with
    the procedural albedo on every surface: the triangles carry the albedo
    at their centroids, the scan an intensity image with N(0, 0.01) noise.
    Depth alone leaves the pose's in-plane translation and its rotation about
    the wall's normal unobservable; color fixes them.  n_poses starts
    N(0, 4 cm) / N(0, 1.5 deg) per axis around the truth."""
    cam = S.QVGA
    scene = S.random_box_room(seed, (4.0, 4.0, 2.5), 0)
    mesh = S.triangulate_scene(scene, cell=cell)
    T = S.look_pose(np.array([2.0, 2.5, 1.25]), np.pi / 2)        # facing the wall y = 4 from 1.5 m
    depth = S.range_image(scene, cam, T, seed + 13, noise_rel=0.005)
    color = S.intensity_image(scene, cam, T, seed + 17, noise=0.01)
    rng = np.random.default_rng(seed)
    poses = np.stack([S.perturb(T, rng, 0.04, np.deg2rad(1.5)) for _ in range(n_poses)])
    return Workload("textured_wall", cam, scene, T, depth, poses, map_mesh=mesh,
                    map_color=S.triangle_albedo(mesh[0], mesh[1]), scan_color=color)

@dataclass
class StreamScan:
    cam: S.Camera
    T_true: np.ndarray                 # [3,4] ground truth of the scan
    depth: np.ndarray                  # [H,W] f32 range image
    poses: np.ndarray                  # [n,3,4] candidate poses


@dataclass
class Stream:
    """Several scans of different resolutions, each with its own candidate
    poses, scored against one map in a single launch."""
    name: str
    scene: S.Scene
    view_cam: S.Camera
    views: list
    view_depths: list
    scans: list
    stride: int = 2
    max_edge: float = 0.1
    smooth_radius: int = 2
    z_min: float = 0.5
    z_max: float = 8.0


def _corridor_pose(x, phase=0.0):
    """Sensor on a walk down the corridor: weaving across it, bobbing, yawing
    about the axis and tilted slightly down."""
    pos = np.array([x, 1.25 + 0.3 * np.sin(x / 3.0 + phase), 1.4 + 0.1 * np.sin(x / 5.0)])
    return S.look_pose(pos, 0.25 * np.sin(x / 4.0 + phase), -0.1)


def uneven(seed: int = 5, n_views: int = 56, n_scans: int = 32) -> Stream:
    """60 m cluttered corridor; map = 56 QVGA views 1 m apart along the walk,
    meshified at stride 2 with smoothing radius 2 (56 x 37,842 = 2,119,152
    triangles); 32 query scans between the views, cycling 320x240, 640x480 and
    1280x960, each with 16-128 candidates N(0, 3 cm) / N(0, 1.5 deg)."""
    scene = S.corridor_scene(seed)
    views = [_corridor_pose(1.0 + k) for k in range(n_views)]
    depths = [S.range_image(scene, S.QVGA, T, seed * 1000 + k, noise_rel=0.01, dropout=0.02)
              for k, T in enumerate(views)]
    rng = np.random.default_rng(seed)
    cams = (S.QVGA, S.KINECT, S.WIDE)
    scans = []
    for j in range(n_scans):
        T = _corridor_pose(1.37 + j * 1.7, phase=0.2)
        cam = cams[j % 3]
        depth = S.range_image(scene, cam, T, seed * 100 + j, noise_rel=0.01, dropout=0.02)
        n = int(rng.integers(16, 129))
        poses = np.stack([S.perturb(T, rng, 0.03, np.deg2rad(1.5)) for _ in range(n)])
        scans.append(StreamScan(cam, T, depth, poses))
    return Stream("uneven", scene, S.QVGA, views, depths, scans)


def _loop_pose(scene, s, frac=0.75, phase=0.0):
    """Sensor on a looped walk around the inside of a room: along the ellipse
    at ``frac`` of the room's half extents (``s`` = arc length, periodic),
    looking inward at a point that wanders around the room centre, with the
    height and pitch varying slowly so that successive laps differ."""
    c = _room_center(scene)
    a, b = frac * 0.5 * (scene.room_hi[0] - scene.room_lo[0]), frac * 0.5 * (scene.room_hi[1] - scene.room_lo[1])
    # arc length of the ellipse by Ramanujan's approximation of its perimeter
    per = np.pi * (3 * (a + b) - np.sqrt((3 * a + b) * (a + 3 * b)))
    ang = 2 * np.pi * (s / per)
    pos = np.array([c[0] + a * np.cos(ang), c[1] + b * np.sin(ang), 1.45 + 0.25 * np.sin(s / 7.3 + phase)])
    tgt = c[:2] + 0.6 * np.array([np.sin(s / 5.1 + phase), np.cos(s / 6.7 + phase)])
    yaw = np.arctan2(tgt[1] - pos[1], tgt[0] - pos[0])
    return S.look_pose(pos, yaw, np.deg2rad(-22.0 + 10.0 * np.sin(s / 4.3 + phase)))


def _range_images(jobs, workers=None):
    """Range images of (scene, cam, T, seed, kwargs) jobs, in a process pool."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    n = workers or min(16, os.cpu_count() or 1)
    if n <= 1 or len(jobs) < 8:
        return [S.range_image(sc, cam, T, seed, **kw) for sc, cam, T, seed, kw in jobs]
    with ProcessPoolExecutor(max_workers=n) as ex:
        futs = [ex.submit(S.range_image, sc, cam, T, seed, **kw) for sc, cam, T, seed, kw in jobs]
        return [f.result() for f in futs]


@dataclass
class Trajectory:
    """A sensor walking a loop through a mapped scene: the map views and, for
    every scan, its ground truth, range image and initial pose estimate."""
    name: str
    scene: S.Scene
    view_cam: S.Camera
    views: list
    view_depths: list
    scans: list                        # StreamScan, poses = [1,3,4] initial estimate
    stride: int = 6
    max_edge: float = 0.1 * 6 / 2
    smooth_radius: int = 4
    z_min: float = 0.5
    z_max: float = 8.0


def trajectory(seed: int = 6, n_scans: int = 500, spacing: float = 0.25, init=(0.10, 5.0),
               workers=None) -> Trajectory:
    """Scan-to-map alignment along a looped walk: an 8 x 6 x 2.8 m office room
    with 24 boxes and a doorway; map = 130 Kinect-like views spread over one
    lap of the walk, meshified at stride 6 with node smoothing radius 4
    (130 x 16,748 = 2,177,240 triangles, free-occupied plus free-unknown);
    ``n_scans`` scans ``spacing`` m apart along the loop (0.5 m/s at 2 Hz,
    about 7.5 laps of ~16.6 m for 500 scans), cycling 320x240, 640x480 and
    1280x960, each starting exactly init[0] m and init[1] degrees from its
    truth in random directions."""
    door = S.Door(axis=0, side=1, lo=(2.0, 0.0), hi=(3.0, 2.1))
    scene = S.random_box_room(seed, (8.0, 6.0, 2.8), 24, doors=[door])
    a, b = 0.75 * 4.0, 0.75 * 3.0
    per = np.pi * (3 * (a + b) - np.sqrt((3 * a + b) * (a + 3 * b)))
    views = [_loop_pose(scene, per * (k + 0.5) / 130, phase=0.9 * k) for k in range(130)]
    rng = np.random.default_rng(seed)
    cams = (S.QVGA, S.KINECT, S.WIDE)
    truths = [_loop_pose(scene, 0.3 + j * spacing, phase=0.0) for j in range(n_scans)]
    kw = dict(noise_rel=0.01, dropout=0.02)
    jobs = [(scene, S.KINECT, T, seed * 1000 + k, kw) for k, T in enumerate(views)]
    jobs += [(scene, cams[j % 3], T, seed * 100000 + j, kw) for j, T in enumerate(truths)]
    imgs = _range_images(jobs, workers)
    scans = []
    for j, T in enumerate(truths):
        T0 = S.perturb(T, rng, init[0], np.deg2rad(init[1]), fixed=True)
        scans.append(StreamScan(cams[j % 3], T, imgs[len(views) + j], T0[None]))
    return Trajectory("trajectory", scene, S.KINECT, views, imgs[:len(views)], scans)


@dataclass
class Sequence:
    """A sensor moving through a scene: ground-truth poses and range images,
    for the sequential depth-image alignment of Sec. V-B."""
    name: str
    cam: S.Camera
    scene: S.Scene
    poses: np.ndarray                  # [N,3,4] ground truth
    depths: list                       # N [H,W] f32 range images
    z_min: float = 0.1
    z_max: float = 8.0


def odometry(seed: int = 9, n_frames: int = 33, step: float = 0.03, noise_rel: float = 0.005,
             dropout: float = 0.02, cam: S.Camera | None = None) -> Sequence:
    """Kinect-like 640x480 frames along an arc at 75% of the half extents of
    a 6x5x2.8 m room with 16 boxes, each frame looking across the room:
    consecutive frames ``step`` metres apart (~1 degree of yaw), with a slow
    height and pitch wave; multiplicative range noise and i.i.d. dropouts."""
    rng = np.random.default_rng(seed)
    cam = S.KINECT if cam is None else cam
    scene = S.random_box_room(seed, (6.0, 5.0, 2.8), 16)
    c = _room_center(scene)
    half = 0.5 * (scene.room_hi - scene.room_lo)
    a, b = 0.75 * half[0], 0.75 * half[1]
    ang0 = rng.uniform(0, 2 * np.pi)
    poses, depths = [], []
    ang = ang0
    for k in range(n_frames):
        pos = np.array([c[0] + a * np.cos(ang), c[1] + b * np.sin(ang), 1.4 + 0.1 * np.sin(0.2 * k)])
        yaw = np.arctan2(c[1] - pos[1], c[0] - pos[0]) + 0.2 * np.sin(0.05 * k)
        T = S.look_pose(pos, yaw, np.deg2rad(-20.0 + 5.0 * np.sin(0.13 * k)))
        poses.append(T)
        depths.append(S.range_image(scene, cam, T, seed * 1000 + k, noise_rel=noise_rel, dropout=dropout))
        # arc length per step: the ellipse's speed at this angle
        ang += step / np.hypot(a * np.sin(ang), b * np.cos(ang))
    return Sequence("odometry", cam, scene, np.stack(poses), depths)
