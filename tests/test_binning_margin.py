"""The binning footprint's margin against the rasterization contract (CPU).

The tile binning uses a cheap float32 footprint of each triangle: the camera
centre rounded to float32 before the subtraction, float32 rotation and
projection, no snapping.  A triangle is binned into every tile its footprint,
widened by a margin, reaches, so the margin has to exceed the distance
between that footprint and the contract's snapped triangle wherever the
latter can cover a pixel.  The margin is a 0.25 px base plus
2^-23 (|t|_1 + 9 max|d|_1) (max(fx, fy) + max(W, H)) / z_min per triangle.
These tests emulate the footprint in numpy and check, on scenes placed up to
1e6 m from the world origin, that every on-screen vertex of the oracle's
contract sub-triangles lies within that margin of the footprint vertex
(unclipped triangles), and that the fixed 2 px margin of a plain float32
footprint would not have covered the far scenes (so the bound is needed).
"""
import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

BASE = 0.25


def _f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _fma32(a, b, c):
    # a * b is exact in float64 for float32 operands; one rounding to float32
    return _f32(a * b + c)


def _footprint(xyz, T, cam):
    """float32 camera-frame vertices and projections as the binning computes
    them, and the per-vertex |d|_1 and |t|_1 of the margin bound."""
    R = _f32(T[:3, :3])
    tf = _f32(T[:3, 3])
    d = _f32(xyz.astype(np.float64) - tf)            # float32 subtraction of float32 values
    V = []
    for i in range(3):                                # camera coordinate i = column i of R
        acc = _f32(R[0, i] * d[:, 0])
        acc = _fma32(R[1, i], d[:, 1], acc)
        acc = _fma32(R[2, i], d[:, 2], acc)
        V.append(acc)
    X, Y, Z = V
    with np.errstate(divide="ignore", invalid="ignore"):
        r = _f32(1.0 / Z)
        u = _fma32(_f32(np.float32(cam.fx) * X), r, np.float32(cam.cx))
        v = _fma32(_f32(np.float32(cam.fy) * Y), r, np.float32(cam.cy))
    return Z, u, v, np.abs(d).sum(1), np.abs(tf).sum()


def _max_excess(mesh, cam, poses, base):
    """Largest (vertex distance - margin) over the on-screen vertices of the
    unclipped contract sub-triangles, and the largest plain vertex distance."""
    xyz, tri = mesh[0], mesh[1]
    zn = np.float32(cam.z_near) * (1.0 - 1e-4)
    worst_excess, worst_dist = -np.inf, 0.0
    for T in poses:
        subs = O.contract_subtriangles(mesh, cam, T)
        Z, u, v, dn, tn = _footprint(xyz, T, cam)
        par = subs[:, 0]
        full = np.all(Z[tri[par]] > cam.z_near * 1.01, axis=1)   # not near-clipped
        if not full.any():
            continue
        t3 = tri[par[full]]
        dm = dn[t3].max(1)
        zmin = np.maximum(Z[t3].min(1), zn)
        # (the kernel divides with the hardware reciprocal, relative error ~2^-22: far inside the factor 2)
        m = base + 2.0 ** -23 * (tn + 9.0 * dm) * (max(cam.fx, cam.fy) + max(cam.width, cam.height)) / zmin
        for k in range(3):
            Xs = subs[full, 1 + 2 * k] / 256.0
            Ys = subs[full, 2 + 2 * k] / 256.0
            dist = np.full(Xs.shape, np.inf)
            for j in range(3):
                vi = t3[:, j]
                dist = np.minimum(dist, np.maximum(np.abs(Xs - u[vi]), np.abs(Ys - v[vi])))
            on = (Xs > -1) & (Xs < cam.width) & (Ys > -1) & (Ys < cam.height)
            if on.any():
                worst_excess = max(worst_excess, float((dist - m)[on].max()))
                worst_dist = max(worst_dist, float(dist[on].max()))
    return worst_excess, worst_dist


def _scene(offset, seed):
    scene = S.random_box_room(seed, (4.0, 4.0, 2.5), 8)
    xyz, tri, cls = S.triangulate_scene(scene, cell=0.1, box_cells=4)
    mesh = ((xyz.astype(np.float64) + offset).astype(np.float32), tri, cls)
    rng = np.random.default_rng(seed + 100)
    poses = []
    for _ in range(3):
        T = np.array(S.look_pose(np.array([rng.uniform(1, 3), rng.uniform(1, 3), rng.uniform(0.8, 1.8)]),
                                 rng.uniform(0, 6.28), rng.uniform(-0.5, 0.5), rng.uniform(-0.3, 0.3)), np.float64)
        T[:3, 3] += offset
        poses.append(T)
    return mesh, poses


@pytest.mark.parametrize("scale", [0.0, 1e3, 1e4, 1e5, 3e5, 1e6])
def test_margin_covers_contract_vertices(scale):
    cam = S.Camera(262.5, 262.5, 79.5, 59.5, 160, 120, z_near=0.1, z_far=16.0)
    offset = scale * np.array([1.0, -0.7, 0.3])
    mesh, poses = _scene(offset, 7)
    excess, dist = _max_excess(mesh, cam, poses, BASE)
    assert excess < 0.0, (scale, excess, dist)
    if scale == 0.0:
        assert dist < 0.01          # near the origin only the snap and the projection rounding remain


def test_fixed_margin_would_not_cover_far_scenes():
    """Sanity check that the far scenes exercise the bound: there the plain
    footprint moves by more than the former fixed 2 px margin."""
    cam = S.Camera(262.5, 262.5, 79.5, 59.5, 160, 120, z_near=0.1, z_far=16.0)
    mesh, poses = _scene(1e6 * np.array([1.0, -0.7, 0.3]), 7)
    _, dist = _max_excess(mesh, cam, poses, BASE)
    assert dist > 2.0
