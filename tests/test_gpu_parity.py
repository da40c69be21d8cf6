"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Every input is seeded and synthetic; every expected value comes from the
oracle.  Sizes: the tiny room at full frame (several tiles plus ragged
edges), the Kinect-like map at 640x480 on sampled pixels, the 1M-triangle
differentiation map at the launch configuration the benchmark times, the
~4M-triangle wide-FOV corridor at 1280x960 with 256 poses per launch, and the
uneven stream of 32 scans of three resolutions against a 2.1M-triangle map,
on sampled pixels.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from workloads import scenes as S

from gpu_helpers import (EPS, compare_records, flagged_pixels, oracle_map, render_mismatch, sample_pixels, stream,
                         stream_map, workload)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_06813_amd as rm
    rm.load_library()
    return rm


DEV = "cuda:0"


def _dev_mesh(rm, mesh):
    return rm.Mesh.from_arrays(*mesh, device=DEV).prepare()


def _T(poses):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(poses).reshape(-1, 12))).to(DEV)


# ------------------------------------------------------------------ scan image / meshify

def test_scan_image_bitexact(rm):
    _say("scan_image")
    rng = np.random.default_rng(0)
    z = rng.uniform(0.0, 10.0, (37, 53)).astype(np.float32)
    z[rng.random(z.shape) < 0.1] = 0.0
    z[rng.random(z.shape) < 0.05] = np.nan
    z[rng.random(z.shape) < 0.05] = np.inf
    z[rng.random(z.shape) < 0.05] = -1.0
    z[0, :4] = [0.5, 8.0, np.float32(0.49999997), np.float32(8.000001)]
    d, c = O.scan_image(z, 0.5, 8.0)
    s = rm.scan_image(torch.from_numpy(z).to(DEV), 0.5, 8.0)
    np.testing.assert_array_equal(s.cls.cpu().numpy(), c)
    np.testing.assert_array_equal(s.depth.cpu().numpy(), d)   # NaN positions compare equal


@pytest.mark.parametrize("stride,radius", [(1, 0), (3, 0), (4, 0), (8, 0), (1, 3), (4, 2), (8, 4)])
def test_meshify_bitexact(rm, stride, radius):
    _say(f"meshify stride {stride} smoothing radius {radius}")
    w = workload("kinect")
    for k in (0, 5):
        depth, T = w.view_depths[k].copy(), w.views[k]
        depth[::97, ::89] = np.nan            # dead pixels drop quads
        xyz, tri, cls = O.meshify(depth, w.cam, T, stride, w.z_min, w.z_max, 0.1 * stride / 2, radius)
        m = rm.mesh_from_range(torch.from_numpy(depth).to(DEV), w.cam, T, stride, w.z_min, w.z_max,
                               0.1 * stride / 2, radius)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(m.xyz.cpu().numpy(), xyz)
        np.testing.assert_array_equal(m.tri.cpu().numpy(), tri)
        np.testing.assert_array_equal(m.cls.cpu().numpy(), cls)


def test_meshify_ragged_and_tiny(rm):
    _say("meshify ragged")
    cam = S.Camera(30.0, 30.0, 9.5, 6.5, 21, 14)
    rng = np.random.default_rng(1)
    T = S.look_pose(np.array([0.3, -0.2, 1.0]), 0.4, 0.1)
    for depth in (rng.uniform(0.4, 9.0, (14, 21)).astype(np.float32), np.zeros((14, 21), np.float32),
                  np.full((14, 21), np.nan, np.float32)):
        for s, rad in ((1, 0), (2, 0), (5, 0), (20, 0), (1, 2), (5, 4)):
            ref = O.meshify(depth, cam, T, s, smooth_radius=rad)
            m = rm.mesh_from_range(torch.from_numpy(depth).to(DEV), cam, T, s, smooth_radius=rad)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(m.xyz.cpu().numpy(), ref[0])
            np.testing.assert_array_equal(m.tri.cpu().numpy(), ref[1])
            np.testing.assert_array_equal(m.cls.cpu().numpy(), ref[2])


# ------------------------------------------------------------------ z-buffer

def _render_cmp(rm, mesh_np, cam, poses, pixels=None, max_flag_frac=0.01):
    dm = _dev_mesh(rm, mesh_np)
    out = rm.render_depth(dm, cam, _T(poses))
    gd = out["depth"].cpu().numpy()
    gt = out["tri"].cpu().numpy()
    gc = out["cls"].cpu().numpy()
    for b, T in enumerate(poses):
        rend = O.render(mesh_np, cam, T, pixels)
        bad, rel, nflag = render_mismatch(rend, cam, gd[b], gt[b])
        assert bad == 0, f"pose {b}: {bad} unflagged id mismatches"
        assert rel <= 1e-5, f"pose {b}: depth rel err {rel}"
        assert nflag <= max_flag_frac * len(rend["pixels"]) + 2
        # class map follows the id map
        gcl = gc[b].reshape(-1)[rend["pixels"]]
        gid = gt[b].reshape(-1)[rend["pixels"]]
        exp = np.where(gid >= 0, mesh_np[2][np.maximum(gid, 0)], O.NONE)
        np.testing.assert_array_equal(gcl, exp)


def test_render_tiny_full_frame(rm):
    _say("render tiny")
    w = workload("tiny")
    rng = np.random.default_rng(3)
    poses = [w.T_true, w.poses[0]] + [S.perturb(w.T_true, rng, 0.3, np.deg2rad(30)) for _ in range(6)]
    _render_cmp(rm, w.map_mesh, w.cam, poses)


def test_render_near_plane_clipping(rm):
    """Poses close to walls and boxes so that many triangles cross z_near."""
    _say("render clip")
    w = workload("tiny")
    cam = S.Camera(52.5, 52.5, 31.5, 23.5, 64, 48, z_near=0.1, z_far=16.0)
    rng = np.random.default_rng(4)
    poses = []
    for k in range(8):
        pos = np.array([rng.uniform(0.05, 0.3), rng.uniform(0.3, 3.7), rng.uniform(0.2, 2.3)])
        poses.append(S.look_pose(pos, rng.uniform(-np.pi, np.pi), rng.uniform(-1.2, 1.2), rng.uniform(-1, 1)))
    _render_cmp(rm, w.map_mesh, cam, poses)


def test_render_ragged_image_and_big_triangles(rm):
    """An image size that is no multiple of any tile, and triangles far
    larger than a tile (the 64-bit edge-function path)."""
    _say("render ragged")
    scene = S.random_box_room(7, (4.0, 4.0, 2.5), 8)
    mesh = S.triangulate_scene(scene, cell=2.0)            # huge wall triangles
    cam = S.Camera(70.0, 70.0, 50.5, 33.5, 101, 67)
    rng = np.random.default_rng(5)
    poses = [S.look_pose(np.array([rng.uniform(1, 3), rng.uniform(1, 3), rng.uniform(0.8, 1.8)]),
                         rng.uniform(0, 6.28), rng.uniform(-0.5, 0.5), rng.uniform(-0.3, 0.3)) for _ in range(6)]
    _render_cmp(rm, mesh, cam, poses)
    for tile in ((16, 16), (64, 32)):
        rm.context().set_tile(*tile)
        try:
            _render_cmp(rm, mesh, cam, poses[:2])
        finally:
            rm.context().set_tile(0, 0)


def test_render_far_from_origin(rm):
    """A room 3e5 m from the world origin, where rounding the camera centre
    to float32 moves the binning footprint by a few pixels: the per-triangle
    binning margin has to cover it, so that no pixel of the contract is lost
    at a tile border (the whole frame is compared, at two tile shapes)."""
    _say("render far from origin")
    scene = S.random_box_room(7, (4.0, 4.0, 2.5), 8)
    xyz, tri, cls = S.triangulate_scene(scene, cell=0.1, box_cells=4)
    off = np.array([3e5, -2.1e5, 0.9e5])
    mesh = ((xyz.astype(np.float64) + off).astype(np.float32), tri, cls)
    cam = S.Camera(262.5, 262.5, 79.5, 59.5, 160, 120, z_near=0.1, z_far=16.0)
    rng = np.random.default_rng(6)
    poses = []
    for _ in range(4):
        T = np.array(S.look_pose(np.array([rng.uniform(1, 3), rng.uniform(1, 3), rng.uniform(0.8, 1.8)]),
                                 rng.uniform(0, 6.28), rng.uniform(-0.5, 0.5), rng.uniform(-0.3, 0.3)), np.float64)
        T[:3, 3] += off
        poses.append(T)
    for tile in ((16, 16), (64, 32)):
        rm.context().set_tile(*tile)
        try:
            _render_cmp(rm, mesh, cam, poses)
        finally:
            rm.context().set_tile(0, 0)


def _layer_stack(seed, n_layers=80, nx=20, ny=16):
    """n_layers tilted, holed rectangles stacked 1.0 .. 3.0 m in front of
    the identity camera, each slightly wider than the 64x48 view at its
    depth, triangle ids shuffled so that every bin mixes the layers."""
    rng = np.random.default_rng(seed)
    xyz, tri = [], []
    for k in range(n_layers):
        z = 1.0 + 2.0 * k / n_layers
        sx, sy = rng.uniform(-0.15, 0.15, size=2)          # depth slopes: layers cross each other
        hx, hy = 0.7 * z, 0.55 * z
        u = np.linspace(-hx, hx, nx + 1)
        v = np.linspace(-hy, hy, ny + 1)
        uu, vv = np.meshgrid(u, v, indexing="ij")
        pts = np.stack([uu, vv, z + sx * uu + sy * vv], -1).reshape(-1, 3)
        idx = np.arange((nx + 1) * (ny + 1)).reshape(nx + 1, ny + 1)
        keep = rng.random((nx, ny)) > 0.25                  # holes show deeper layers through
        q00, q01 = idx[:-1, :-1][keep], idx[:-1, 1:][keep]
        q10, q11 = idx[1:, :-1][keep], idx[1:, 1:][keep]
        off = sum(len(p) for p in xyz)
        tri.append(np.concatenate([np.stack([q00, q01, q11], 1), np.stack([q00, q11, q10], 1)]) + off)
        xyz.append(pts)
    xyz = np.concatenate(xyz).astype(np.float32)
    tri = np.concatenate(tri).astype(np.int32)
    tri = tri[rng.permutation(len(tri))]
    return xyz, tri, np.zeros(len(tri), np.uint8)


def test_render_deep_stack_many_rounds(rm):
    """About 38,000 triangles in 80 crossing, holed layers over a 64x48 view,
    in shuffled order: tile bins take tens of rounds, so the depth
    snapshot's refresh schedule (every round at first, then every few) and
    the occlusion skips it drives decide most triangles.  Full-frame parity
    with the oracle at three tile shapes and five poses."""
    _say("render deep stack")
    mesh = _layer_stack(23)
    cam = S.Camera(52.5, 52.5, 31.5, 23.5, 64, 48, z_near=0.1, z_far=16.0)
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    rng = np.random.default_rng(29)
    poses = [T] + [S.perturb(T, rng, 0.05, np.deg2rad(3)) for _ in range(4)]
    for tile in ((64, 32), (16, 16), (8, 8)):
        rm.context().set_tile(*tile)
        try:
            _render_cmp(rm, mesh, cam, poses)
        finally:
            rm.context().set_tile(0, 0)


def _big_overlap(seed, n=900):
    """n large triangles over the 64x48 view of the identity camera, at
    random depths 0.6 .. 3.0 m, each spanning most of the view; every third
    has one vertex, every ninth two, in front of the near plane (down to
    behind the camera, off to a side), so that it is clipped into two
    sub-triangles or one.
    Triangle ids shuffled."""
    rng = np.random.default_rng(seed)
    pts = []
    for k in range(n):
        z = rng.uniform(0.6, 3.0, size=3)
        ang = rng.uniform(0, 2 * np.pi) + np.array([0.0, 2.1, 4.2]) + rng.uniform(-0.3, 0.3, 3)
        r = rng.uniform(0.6, 1.1, 3)
        x, y = 0.6 * r * np.cos(ang) * z, 0.45 * r * np.sin(ang) * z
        side = rng.choice([-1.0, 1.0])
        for j in range(1 + (k % 9 == 0) if k % 3 == 0 else 0):
            # off to one side, so that the part near the camera leaves the view
            z[j] = rng.uniform(-0.3, 0.08)
            x[j], y[j] = side * rng.uniform(0.6, 1.0), rng.uniform(-0.3, 0.3)
        pts.append(np.stack([x, y, z], 1))
    xyz = np.concatenate(pts).astype(np.float32)
    tri = np.arange(3 * n, dtype=np.int32).reshape(n, 3)[rng.permutation(n)]
    return xyz, tri, np.zeros(n, np.uint8)


def test_render_band_queue_overflow(rm):
    """900 large, overlapping triangles over one 64x48 view: the first round
    of a tile offers 256 of them, every one above the in-thread size and none
    culled yet, so more sub-triangles ask for the band queue than it holds
    and the round takes further queue passes; near-plane crossings split
    triangles in two, so some threads come back with only their second
    sub-triangle.  Full-frame parity with the oracle at three tile shapes."""
    _say("render band queue overflow")
    mesh = _big_overlap(31)
    cam = S.Camera(52.5, 52.5, 31.5, 23.5, 64, 48, z_near=0.1, z_far=16.0)
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    rng = np.random.default_rng(37)
    poses = [T] + [S.perturb(T, rng, 0.05, np.deg2rad(3)) for _ in range(3)]
    for tile in ((64, 32), (32, 32), (16, 16)):
        rm.context().set_tile(*tile)
        try:
            _render_cmp(rm, mesh, cam, poses)
        finally:
            rm.context().set_tile(0, 0)


def test_cost_grad_band_queue_overflow(rm):
    """Cost, gradient and Gauss-Newton blocks through the rounds that take
    further band-queue passes: the 900 overlapping triangles against a scan
    the oracle renders from a nearby pose, four poses, at two tile shapes,
    against the oracle's reduction over its unflagged pixels."""
    _say("cost+grad band queue overflow")
    mesh = _big_overlap(31)
    cam = S.Camera(52.5, 52.5, 31.5, 23.5, 64, 48, z_near=0.1, z_far=16.0)
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    rng = np.random.default_rng(41)
    rend = O.render(mesh, cam, S.perturb(T, rng, 0.02, np.deg2rad(1)), None)
    depth = np.zeros(cam.width * cam.height, np.float32)
    hit = rend["id"] >= 0
    depth[rend["pixels"][hit]] = rend["z"][hit]
    depth = depth.reshape(cam.height, cam.width)
    poses = [T] + [S.perturb(T, rng, 0.03, np.deg2rad(2)) for _ in range(3)]
    for tile in ((64, 32), (16, 16)):
        rm.context().set_tile(*tile)
        try:
            _cost_case_scan(rm, mesh, cam, depth, 0.05, 8.0, poses, None)
        finally:
            rm.context().set_tile(0, 0)


def test_duplicate_triangles_lowest_id_wins(rm):
    """Every triangle of the tiny room twice, the two copies at shuffled
    positions (ids): at every pixel the GPU's triangle id is the lower id of
    the two copies of the triangle the oracle sees there.  The copies tie
    exactly, so this is checked directly, without the near-tie exemption;
    only pixels where two different triangles of the original mesh nearly
    tie are left out."""
    _say("render duplicate triangles")
    w = workload("tiny")
    xyz, tri, cls = w.map_mesh
    n = len(tri)
    rng = np.random.default_rng(17)
    pos = rng.permutation(2 * n)                 # copy a of t at pos[2t], copy b at pos[2t+1]
    tri2 = np.empty((2 * n, 3), np.int32)
    cls2 = np.empty(2 * n, np.uint8)
    tri2[pos[0::2]] = tri; tri2[pos[1::2]] = tri
    cls2[pos[0::2]] = cls; cls2[pos[1::2]] = cls
    low = np.minimum(pos[0::2], pos[1::2])
    dm = _dev_mesh(rm, (xyz, tri2, cls2))
    poses = [w.T_true, w.poses[0]] + [S.perturb(w.T_true, rng, 0.3, np.deg2rad(30)) for _ in range(4)]
    out = rm.render_depth(dm, w.cam, _T(poses))
    gt = out["tri"].cpu().numpy()
    for b, T in enumerate(poses):
        rend = O.render(w.map_mesh, w.cam, T)
        fl = O.flags(rend, w.cam)
        ok = ~(fl["near_tie"] | fl["far_tie"])
        exp = np.where(rend["id"] >= 0, low[np.maximum(rend["id"], 0)], -1)
        got = gt[b].reshape(-1)
        assert ok.mean() > 0.97
        np.testing.assert_array_equal(got[ok], exp[ok])
        # the oracle on the duplicated mesh agrees: lower copy, exact tie
        rend2 = O.render((xyz, tri2, cls2), w.cam, T)
        np.testing.assert_array_equal(rend2["id"][ok], exp[ok])
        hit = ok & (rend2["id"] >= 0)
        np.testing.assert_array_equal(rend2["z2"][hit], rend2["z"][hit])


def test_render_kinect_sampled(rm):
    _say("render kinect")
    w = workload("kinect")
    mesh = oracle_map("kinect")
    pix = sample_pixels(w.cam, 3000, 11)
    _render_cmp(rm, mesh, w.cam, list(w.poses[:4]), pixels=pix)


def test_render_empty_mesh_and_pointing_away(rm):
    _say("render empty")
    w = workload("tiny")
    empty = (np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.zeros(0, np.uint8))
    dm = rm.Mesh.from_arrays(*empty, device=DEV)
    out = rm.render_depth(dm, w.cam, _T([w.T_true]))
    assert (out["tri"].cpu().numpy() == -1).all()
    assert np.isnan(out["depth"].cpu().numpy()).all()
    # a camera outside the room looking away sees nothing
    T = S.look_pose(np.array([2.0, -3.0, 1.2]), -np.pi / 2)
    out = rm.render_depth(_dev_mesh(rm, w.map_mesh), w.cam, _T([T]))
    assert (out["cls"].cpu().numpy() == rm.NONE).all()


# ------------------------------------------------------------------ cost and gradient

def _cost_case(rm, name, poses, pixels, grad=True, mesh_np=None):
    w = workload(name)
    mesh_np = oracle_map(name) if mesh_np is None else mesh_np
    return _cost_case_scan(rm, mesh_np, w.cam, w.scan_depth, w.z_min, w.z_max, poses, pixels, grad)


def _cost_case_scan(rm, mesh_np, cam, scan_depth, z_min, z_max, poses, pixels, grad=True, dm=None):
    """GPU records of single-pose launches restricted (by the scan mask) to
    the sampled pixels the oracle does not flag, against the oracle's
    reduction over the same pixels."""
    d, c = O.scan_image(scan_depth, z_min, z_max)
    dm = _dev_mesh(rm, mesh_np) if dm is None else dm
    scan = rm.scan_image(torch.from_numpy(scan_depth).to(DEV), z_min, z_max, cam=cam)
    res = []
    masks = []
    for b, T in enumerate(poses):
        rend = O.render(mesh_np, cam, T, pixels)
        terms = O.pixel_terms(rend, mesh_np[2], d, c, cam, EPS)
        flagged = flagged_pixels(rend, terms, cam, EPS)
        keep = ~flagged
        ref = O.reduce_terms(terms, keep)
        mask = np.zeros(cam.width * cam.height, np.uint8)
        mask[rend["pixels"][keep]] = 1
        masks.append(mask)
        res.append((ref, terms, keep))
    outs = []
    for b, T in enumerate(poses):
        scan.mask = torch.from_numpy(masks[b].reshape(cam.height, cam.width)).to(DEV)
        f = rm.align_cost_grad if grad else rm.align_cost
        outs.append(f(dm, scan, _T([T]), EPS).cpu().numpy()[0])
    for b in range(len(poses)):
        ref, terms, keep = res[b]
        compare_records(outs[b], ref, terms, keep, EPS, grad=grad)
        assert keep.mean() > 0.95
    return outs


def test_cost_grad_tiny_full_frame(rm):
    _say("cost tiny")
    w = workload("tiny")
    rng = np.random.default_rng(6)
    poses = [w.T_true, w.poses[0]] + [S.perturb(w.T_true, rng, 0.05, np.deg2rad(3)) for _ in range(4)]
    _cost_case(rm, "tiny", poses, None)
    _cost_case(rm, "tiny", poses[:2], None, grad=False)


def test_cost_grad_kinect_sampled(rm):
    _say("cost kinect")
    w = workload("kinect")
    _cost_case(rm, "kinect", list(w.poses[:3]), sample_pixels(w.cam, 4000, 12))


@pytest.mark.slow
def test_cost_grad_differentiation_1m_sampled(rm):
    """The 1M-triangle map at 640x480 in the benchmark's launch configuration:
    one B = 64 launch (default tile, persistent schedule).  Rows of that
    launch equal single-pose launches, and the same B = 64 launch restricted
    (by the scan mask) to sampled pixels that none of three compared poses
    flags matches the oracle's reduction over those pixels for each of them."""
    _say("cost differentiation (1M triangles, B = 64)")
    w = workload("differentiation")
    mesh = oracle_map("differentiation")
    dm = _dev_mesh(rm, mesh)
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), w.z_min, w.z_max, cam=w.cam)
    T = _T(w.poses)
    assert T.shape[0] == 64
    allr = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    picks = (0, 31, 63)
    for i in picks:
        one = rm.align_cost_grad(dm, scan, T[i:i + 1].contiguous(), EPS).cpu().numpy()
        np.testing.assert_array_equal(one[0], allr[i])
    pix = sample_pixels(w.cam, 1500, 13)
    d, c = O.scan_image(w.scan_depth, w.z_min, w.z_max)
    cases, keep = [], np.ones(len(pix), bool)
    for i in picks:
        rend = O.render(mesh, w.cam, w.poses[i], pix)
        terms = O.pixel_terms(rend, mesh[2], d, c, w.cam, EPS)
        keep &= ~flagged_pixels(rend, terms, w.cam, EPS)
        cases.append(terms)
    assert keep.mean() > 0.9
    mask = np.zeros(w.cam.width * w.cam.height, np.uint8)
    mask[pix[keep]] = 1
    scan.mask = torch.from_numpy(mask.reshape(w.cam.height, w.cam.width)).to(DEV)
    masked = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    for i, terms in zip(picks, cases):
        compare_records(masked[i], O.reduce_terms(terms, keep), terms, keep, EPS)


@pytest.mark.slow
def test_cost_grad_wide_4m_full_batch(rm):
    """Wide-FOV corridor: 1280x960, ~4M triangles, 10% dead pixels, 256 poses
    in one launch.  Rows of the full launch equal single-pose launches, and
    sampled pixels of two poses match the oracle."""
    _say("cost wide (4M triangles, 256 poses)")
    w = workload("wide")
    mesh = oracle_map("wide")
    dm = _dev_mesh(rm, mesh)
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), w.z_min, w.z_max, cam=w.cam)
    T = _T(w.poses)
    allr = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    assert allr.shape[0] == 256
    for i in (0, 131, 255):
        one = rm.align_cost_grad(dm, scan, T[i:i + 1].contiguous(), EPS).cpu().numpy()
        np.testing.assert_array_equal(one[0], allr[i])
    _cost_case_scan(rm, mesh, w.cam, w.scan_depth, w.z_min, w.z_max, list(w.poses[:2]),
                    sample_pixels(w.cam, 800, 14), dm=dm)


@pytest.mark.slow
def test_uneven_stream_full_shape(rm):
    """32 scans of 320x240, 640x480 and 1280x960 with 16-128 poses each in one
    launch against the 2.1M-triangle corridor map: rows equal one launch per
    scan, and sampled pixels of one pose per resolution match the oracle."""
    _say("uneven stream (32 scans, 2.1M triangles)")
    st = stream("uneven")
    mesh = stream_map("uneven")
    dm = _dev_mesh(rm, mesh)
    scans = [rm.scan_image(torch.from_numpy(s.depth).to(DEV), st.z_min, st.z_max, cam=s.cam) for s in st.scans]
    counts = [len(s.poses) for s in st.scans]
    T = _T(np.concatenate([s.poses for s in st.scans]))
    allr = rm.align_cost_grad(dm, scans, T, EPS, poses_per_scan=counts).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(counts)])
    for k in (0, 1, 2, 31):
        sep = rm.align_cost_grad(dm, scans[k], T[off[k]:off[k + 1]].contiguous(), EPS).cpu().numpy()
        np.testing.assert_array_equal(sep, allr[off[k]:off[k + 1]])
    for k in (0, 1, 2):
        s = st.scans[k]
        _cost_case_scan(rm, mesh, s.cam, s.depth, st.z_min, st.z_max, [s.poses[0]],
                        sample_pixels(s.cam, 600, 20 + k), dm=dm)


def test_unmasked_totals_within_flag_bound(rm):
    """Without a mask, totals differ from the oracle only through flagged pixels."""
    _say("unmasked totals")
    w = workload("tiny")
    d, c = O.scan_image(w.scan_depth)
    dm = _dev_mesh(rm, w.map_mesh)
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    g = rm.align_cost_grad(dm, scan, _T(w.poses), EPS).cpu().numpy()[0]
    ref = O.align_cost(w.map_mesh, w.cam, w.poses[0], d, c, eps=EPS)
    nflag = flagged_pixels(ref["render"], ref["terms"], w.cam, EPS).sum()
    assert abs(g[0] - ref["e_table"]) <= 2 * nflag
    assert abs(g[1] - ref["e_soft"]) <= 1e-4 * np.abs(ref["terms"]["rho"]).sum() + 2 * nflag


def test_empty_and_degenerate_costs(rm):
    _say("degenerate costs")
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    nan_scan = rm.scan_image(torch.full((w.cam.height, w.cam.width), float("nan"), device=DEV), cam=w.cam)
    out = rm.align_cost_grad(dm, nan_scan, _T(w.poses), EPS).cpu().numpy()[0]
    assert out[0] == 0 and out[1] == 0 and out[2 + 6] == w.cam.width * w.cam.height
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    empty = rm.Mesh.from_arrays(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), np.zeros(0, np.uint8),
                                device=DEV)
    out = rm.align_cost_grad(empty, scan, _T(w.poses), EPS).cpu().numpy()[0]
    assert out[0] == 0 and out[1] == 0 and out[2 + 7] == w.cam.width * w.cam.height
    T = S.look_pose(np.array([2.0, -3.0, 1.2]), -np.pi / 2)
    out = rm.align_cost_grad(dm, scan, _T([T]), EPS).cpu().numpy()[0]
    assert out[0] == 0 and out[rm.OUT_N_ACTIVE] == 0 and not out[rm.OUT_GRAD:rm.OUT_GRAD + 6].any()


# ------------------------------------------------------------------ invariances

def test_batch_tile_and_run_invariance(rm):
    """Pose i of a batch equals pose i alone; every tile shape and a repeated
    run give bit-identical records."""
    _say("invariance")
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    T = _T(w.poses[:16])
    base = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    again = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    np.testing.assert_array_equal(base, again)
    for i in (0, 7, 15):
        one = rm.align_cost_grad(dm, scan, T[i:i + 1].contiguous(), EPS).cpu().numpy()
        np.testing.assert_array_equal(one[0], base[i])
    ctx = rm.context()
    try:
        for tile in ((8, 8), (16, 16), (32, 32), (64, 32)):
            ctx.set_tile(*tile)
            o = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
            # integer fields identical; float sums reassociate across tiles
            np.testing.assert_array_equal(o[:, [0] + list(range(2, 12))], base[:, [0] + list(range(2, 12))])
            l1 = np.abs(base[:, 1]) + 1
            assert (np.abs(o[:, 1] - base[:, 1]) <= 1e-5 * l1 + 1e-3).all()
            np.testing.assert_allclose(o[:, 18:45], base[:, 18:45], rtol=1e-4, atol=1e-6 * np.abs(base[:, 18:45]).max())
            ro = rm.render_depth(dm, w.cam, T[:2].contiguous())
            ctx.set_tile(0, 0)
            rb = rm.render_depth(dm, w.cam, T[:2].contiguous())
            np.testing.assert_array_equal(ro["tri"].cpu().numpy(), rb["tri"].cpu().numpy())
            np.testing.assert_array_equal(ro["depth"].cpu().numpy(), rb["depth"].cpu().numpy())
    finally:
        ctx.set_tile(0, 0)


def _records_close(o, base):
    """Integer fields equal; float sums equal up to the reassociation of
    per-tile partial sums."""
    ints = [0] + list(range(2, 12)) + [45]
    np.testing.assert_array_equal(o[:, ints], base[:, ints])
    l1 = np.abs(base[:, 1]) + 1
    assert (np.abs(o[:, 1] - base[:, 1]) <= 1e-5 * l1 + 1e-3).all()
    np.testing.assert_allclose(o[:, 18:45], base[:, 18:45], rtol=1e-4, atol=1e-6 * np.abs(base[:, 18:45]).max())


def _plans(text):
    """(bin capacity, spill-list entries, region entries, bins that spill,
    list entries and region entries they need) of each sizing pass in RM_LOG
    output."""
    import re
    pat = re.compile(r"bin capacity (\d+) \(\d+ for large footprints; largest fills \d+ small, \d+ large\), "
                     r"overflow list (\d+) and regions (\d+) entries \((\d+) bins spill; they need (\d+) list "
                     r"and (\d+) region entries\)")
    return [tuple(int(x) for x in m.groups()) for m in pat.finditer(text)]


def test_bin_capacity_override_takes_the_overflow_path(rm, capfd, monkeypatch):
    """rm_set_bin_cap fixes the tile-bin capacity: at 1 entry every bin with
    more than one triangle overflows, at 16 and 256 entries some do.  The
    entries past a bin's capacity spill to the overflow regions (adaptive by
    default), or, with no overflow or when a small fixed one is full, the
    tile is rasterized from every visible cluster of its pose.  Records are
    bit-identical to the adaptive capacity on every path, eagerly and
    replayed from captured graphs, the sizing pass reports the overflow it
    used, and the defaults are restored afterwards."""
    _say("bin capacity override")
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    T = _T(w.poses[:16])
    base = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    ctx = rm.context()
    with pytest.raises(rm.RenderMapError):
        ctx.set_bin_cap(-1)
    with pytest.raises(rm.RenderMapError):
        ctx.set_bin_pool(-2)
    monkeypatch.setenv("RM_LOG", "1")
    try:
        for cap in (1, 16, 256):
            ctx.set_bin_cap(cap)
            for pool in (0, -1, 4096):
                ctx.set_bin_pool(pool)
                capfd.readouterr()
                o = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
                plans = _plans(capfd.readouterr().err)
                _say(f"cap {cap} pool {pool}: sizing passes {plans}")
                np.testing.assert_array_equal(o, base)
                assert plans and all(p[0] == cap for p in plans)
                bc, lst, regs, nrec, spilled, filled = plans[-1]
                assert nrec > 0 and spilled > 0 and filled > 0          # some bins overflow at these capacities
                if pool == 0:
                    assert lst == 0 and regs == 0
                elif pool == -1:
                    assert lst >= spilled and regs >= filled            # every overflowing bin has a region
                else:
                    assert lst == pool and regs == pool
                # a second call of the shape (sized; asynchronous adaptation only)
                np.testing.assert_array_equal(rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy(), base)
            rd = rm.render_depth(dm, w.cam, T[:2].contiguous())
            ctx.set_bin_cap(0)
            rb = rm.render_depth(dm, w.cam, T[:2].contiguous())
            ctx.set_bin_cap(cap)
            np.testing.assert_array_equal(rd["tri"].cpu().numpy(), rb["tri"].cpu().numpy())
        ctx.set_bin_cap(1)
        for pool in (-1, 0):
            ctx.set_bin_pool(pool)
            out = torch.empty((16, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
            rm.align_cost_grad(dm, scan, T, EPS, out=out)
            torch.cuda.synchronize()
            g = rm.Graph(DEV)
            with g:
                rm.align_cost_grad(dm, scan, T, EPS, out=out)
            for _ in range(3):
                out.zero_()
                g.replay()
                junk = torch.randn(1000, device=DEV).sum()
                torch.cuda.synchronize()
                np.testing.assert_array_equal(out.cpu().numpy(), base)
                del junk
            del g
    finally:
        ctx.set_bin_cap(0)
        ctx.set_bin_pool(-1)
    np.testing.assert_array_equal(rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy(), base)


@pytest.mark.slow
def test_uneven_stream_overflow_pool(rm, capfd, monkeypatch):
    """The uneven stream of 32 scans (2,522 poses, 320x240 to 1280x960, 2.1M
    triangles): the bin capacity its 712,110 (pose, tile) records can take in
    the budget is far below its fullest bins, whose excess spills to overflow
    regions.  Records equal those of the every-cluster path (no overflow) and
    of an overflow too small for all of them, bit for bit."""
    _say("uneven stream, overflow pool")
    st = stream("uneven")
    dms = _dev_mesh(rm, stream_map("uneven"))
    scans = [rm.scan_image(torch.from_numpy(x.depth).to(DEV), st.z_min, st.z_max, cam=x.cam) for x in st.scans]
    counts = [len(x.poses) for x in st.scans]
    Ts = _T(np.concatenate([x.poses for x in st.scans]))
    ctx = rm.context()
    ctx.set_tile(64, 32)
    monkeypatch.setenv("RM_LOG", "1")
    try:
        capfd.readouterr()
        got = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
        plans = _plans(capfd.readouterr().err)
        _say(f"sizing passes {plans}")
        bc, lst, regs, nrec, spilled, filled = plans[-1]
        assert nrec > 0 and lst >= spilled > 0 and regs >= filled
        again = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
        np.testing.assert_array_equal(again, got)
        ctx.set_bin_pool(filled // 3)
        part = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
        ctx.set_bin_pool(0)
        none = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
    finally:
        ctx.set_bin_pool(-1)
        ctx.set_tile(0, 0)
    np.testing.assert_array_equal(part, got)
    np.testing.assert_array_equal(none, got)


@pytest.mark.slow
def test_autotune_wide_4m_and_uneven_stream(rm):
    """The tile autotuner on the shapes that need more than 2,048 tiles of
    the small candidates: the 4M-triangle 1280x960 launch of 256 poses and
    the uneven stream of 32 scans (320x240 to 1280x960, 2.1M triangles).  It
    picks one of the four shapes and keeps it for the shape, and the records
    equal those of the fixed 64x32 tile (integer fields exactly, sums up to
    the reassociation of tile partial sums)."""
    _say("autotune (wide 4M, uneven stream)")
    ctx = rm.context()
    w = workload("wide")
    dm = _dev_mesh(rm, oracle_map("wide"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), w.z_min, w.z_max, cam=w.cam)
    T = _T(w.poses)
    st = stream("uneven")
    dms = _dev_mesh(rm, stream_map("uneven"))
    scans = [rm.scan_image(torch.from_numpy(x.depth).to(DEV), st.z_min, st.z_max, cam=x.cam) for x in st.scans]
    counts = [len(x.poses) for x in st.scans]
    Ts = _T(np.concatenate([x.poses for x in st.scans]))
    ctx.set_tile(64, 32)
    base_w = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    base_s = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
    ctx.set_tile(0, 0)
    try:
        ctx.autotune(True)
        got_w = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
        tile_w = ctx.get_tile(w.cam.width, w.cam.height, 256, dm.n_tris)
        got_s = rm.align_cost_grad(dms, scans, Ts, EPS, poses_per_scan=counts).cpu().numpy()
        again = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
    finally:
        ctx.autotune(False)
    _say(f"autotuned tile at 1280x960: {tile_w}")
    assert tile_w in ((64, 32), (32, 32), (16, 16), (8, 8))
    _records_close(got_w, base_w)
    _records_close(got_s, base_s)
    np.testing.assert_array_equal(again, got_w)


def test_tile_limits(rm):
    """8x8 tiles on a 4096-pixel-wide image need 512 tiles per row: the call
    is refused before anything runs; 16x16 tiles (256 per row) are accepted."""
    _say("tile limits")
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    cam = S.Camera(2000.0, 2000.0, 2047.5, 5.5, 4096, 12)
    ctx = rm.context()
    try:
        ctx.set_tile(8, 8)
        with pytest.raises(rm.RenderMapError) as ex:
            rm.render_depth(dm, cam, _T([w.T_true]))
        assert ex.value.code == rm.RM_ERR_UNSUPPORTED
        ctx.set_tile(16, 16)
        a = rm.render_depth(dm, cam, _T([w.T_true]))
        ctx.set_tile(64, 32)
        b = rm.render_depth(dm, cam, _T([w.T_true]))
        np.testing.assert_array_equal(a["tri"].cpu().numpy(), b["tri"].cpu().numpy())
    finally:
        ctx.set_tile(0, 0)


def test_multi_scan_uneven_batch(rm):
    """Scans of different resolutions with uneven pose counts in one launch
    give the same records as one launch per scan."""
    _say("multi-scan")
    wk = workload("kinect")
    mesh = oracle_map("kinect")
    dm = _dev_mesh(rm, mesh)
    cams = [S.QVGA, S.KINECT, S.Camera(400.0, 400.0, 249.5, 149.5, 500, 300), S.TINY]
    rng = np.random.default_rng(9)
    scans, poses, counts = [], [], []
    for k, cam in enumerate(cams):
        depth = S.range_image(wk.scene, cam, wk.T_true, 50 + k, dropout=0.02)
        scans.append(rm.scan_image(torch.from_numpy(depth).to(DEV), cam=cam))
        n = [3, 1, 5, 2][k]
        counts.append(n)
        poses += [S.perturb(wk.T_true, rng, 0.03, np.deg2rad(1.5)) for _ in range(n)]
    T = _T(poses)
    allr = rm.align_cost_grad(dm, scans, T, EPS, poses_per_scan=counts).cpu().numpy()
    off = 0
    for k in range(len(cams)):
        sep = rm.align_cost_grad(dm, scans[k], T[off:off + counts[k]].contiguous(), EPS).cpu().numpy()
        np.testing.assert_array_equal(sep, allr[off:off + counts[k]])
        off += counts[k]
    # and against the oracle for the smallest scan, full frame
    d, c = O.scan_image(S.range_image(wk.scene, S.TINY, wk.T_true, 53, dropout=0.02))
    ref = O.align_cost(mesh, S.TINY, poses[-1], d, c, eps=EPS)
    assert abs(allr[-1][0] - ref["e_table"]) <= 2 * flagged_pixels(ref["render"], ref["terms"], S.TINY, EPS).sum()


def test_schedules_give_identical_records(rm):
    """One workgroup per item, persistent longest-first and automatic
    scheduling give bit-identical records, for one scan and for an uneven
    multi-scan batch; a captured persistent launch replays identically."""
    _say("schedules")
    wk = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(wk.scan_depth).to(DEV), cam=wk.cam)
    T = _T(wk.poses[:24])
    cams = [S.QVGA, S.KINECT, S.Camera(400.0, 400.0, 249.5, 149.5, 500, 300)]
    scans = [rm.scan_image(torch.from_numpy(S.range_image(wk.scene, c, wk.T_true, 60 + k, dropout=0.02)).to(DEV),
                           cam=c) for k, c in enumerate(cams)]
    counts = [7, 13, 4]
    ctx = rm.context()
    res = {}
    try:
        for mode in (1, 2, 0):
            ctx.set_schedule(mode)
            one = rm.align_cost_grad(dm, scan, T, EPS).cpu().numpy()
            multi = rm.align_cost_grad(dm, scans, T, EPS, poses_per_scan=counts).cpu().numpy()
            res[mode] = (one, multi)
        for mode in (2, 0):
            np.testing.assert_array_equal(res[mode][0], res[1][0])
            np.testing.assert_array_equal(res[mode][1], res[1][1])
        ctx.set_schedule(2)
        out = torch.empty((24, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
        rm.align_cost_grad(dm, scans, T, EPS, poses_per_scan=counts, out=out)
        torch.cuda.synchronize()
        g = rm.Graph(DEV)
        with g:
            rm.align_cost_grad(dm, scans, T, EPS, poses_per_scan=counts, out=out)
        for _ in range(3):
            out.zero_()
            g.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), res[1][1])
    finally:
        ctx.set_schedule(0)


# ------------------------------------------------------------------ optimizer step, autograd, graphs

def test_gn_step_and_retract_match_oracle(rm):
    _say("gn step")
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    T = _T(w.poses)
    out = rm.align_cost_grad(dm, scan, T, 0.5)
    o = out.cpu().numpy()[0]
    H = np.zeros((6, 6)); H[np.triu_indices(6)] = o[24:45]; H = H + H.T - np.diag(np.diag(H))
    ref = O.gn_step({"jtj": H, "jtr": o[18:24]}, lam=0.1)
    T2 = T.clone()
    delta = torch.empty((1, 6), dtype=torch.float64, device=DEV)
    rm.gn_step(out, T2, 0.1, delta)
    np.testing.assert_allclose(delta.cpu().numpy()[0], ref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(T2.cpu().numpy().reshape(3, 4), O.retract(w.poses[0], ref), atol=1e-12)
    rng = np.random.default_rng(0)
    dl = rng.normal(size=(5, 6)) * np.array([0.1, 0.1, 0.1, 0.5, 0.5, 0.5])
    dl[0, 3:] = 1e-9
    Ts = np.stack([S.perturb(w.T_true, rng, 0.5, 0.5) for _ in range(5)])
    got = rm.se3_retract(_T(Ts), torch.from_numpy(dl).to(DEV)).cpu().numpy().reshape(5, 3, 4)
    for k in range(5):
        np.testing.assert_allclose(got[k], O.retract(Ts[k], dl[k]), atol=1e-13)


def test_adam_step_matches_oracle(rm):
    """rm_adam_step over five consecutive steps of 9 poses, with gradients,
    moments and poses of widely different scales: moments, increments and
    poses match the oracle's Adam update and retraction."""
    _say("adam step")
    rng = np.random.default_rng(31)
    P = 9
    w = workload("tiny")
    Ts = np.stack([S.perturb(w.T_true, rng, 0.5, 0.5) for _ in range(P)])
    T = _T(Ts)
    m = torch.zeros((P, 6), dtype=torch.float64, device=DEV)
    v = torch.zeros((P, 6), dtype=torch.float64, device=DEV)
    mo, vo, To = np.zeros((P, 6)), np.zeros((P, 6)), Ts.reshape(P, 3, 4).copy()
    for step in range(1, 6):
        g = rng.normal(size=(P, 6)) * 10.0 ** rng.uniform(-4, 3, (P, 6))
        g[0] = 0.0                                   # a zero gradient: the guard keeps the step finite
        rec = np.zeros((P, rm.OUT_STRIDE))
        rec[:, rm.OUT_GRAD:rm.OUT_GRAD + 6] = g
        lr, b1, b2 = 0.02 / step, 0.85, 0.99
        rm.adam_step(torch.from_numpy(rec).to(DEV), T, m, v, step, lr, b1, b2)
        for p in range(P):
            d, mo[p], vo[p] = O.adam_step(g[p], mo[p], vo[p], step, lr, b1, b2)
            To[p] = O.retract(To[p], d)
        np.testing.assert_allclose(m.cpu().numpy(), mo, rtol=1e-13, atol=0)
        np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=1e-13, atol=0)
        np.testing.assert_allclose(T.cpu().numpy().reshape(P, 3, 4), To, rtol=0, atol=1e-12)
    with pytest.raises(ValueError):
        rm.adam_step(torch.zeros((P - 1, rm.OUT_STRIDE), dtype=torch.float64, device=DEV), T, m, v, 6, 0.01)
    with pytest.raises(ValueError):
        rm.adam_step(torch.zeros((P, rm.OUT_STRIDE), dtype=torch.float64, device=DEV), T, m[:-1], v, 6, 0.01)


def _tiny_masked_scan(rm, w, mask):
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    scan.mask = torch.from_numpy(mask.reshape(w.cam.height, w.cam.width).astype(np.uint8)).to(DEV)
    return scan


def test_autograd_function_matches_oracle_gradient(rm):
    """AlignCost (the autograd.Function) over the pixels the oracle does not
    flag: its value and gradient match the oracle within 1e-4 of their L1
    mass."""
    _say("autograd")
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    d, c = O.scan_image(w.scan_depth)
    ref_all = O.align_cost(w.map_mesh, w.cam, w.poses[0], d, c, eps=EPS)
    t = ref_all["terms"]
    keep = ~flagged_pixels(ref_all["render"], t, w.cam, EPS)
    assert keep.mean() > 0.95
    ref = O.reduce_terms(t, keep)
    scan = _tiny_masked_scan(rm, w, keep)
    T0 = _T(w.poses)
    delta = torch.zeros((1, 6), dtype=torch.float64, device=DEV, requires_grad=True)
    e = rm.AlignCost.apply(delta, T0, dm, scan, EPS)
    (2.0 * e.sum()).backward()
    l1 = max(np.abs(t["rho"][keep]).sum(), 1.0)
    assert abs(e.item() - ref["e_soft"]) <= 1e-4 * l1, (e.item(), ref["e_soft"])
    gl1 = (4.0 / EPS ** 2) * np.abs(t["r"][keep, None] * t["J"][keep]).sum(0)
    g = delta.grad.cpu().numpy()[0] / 2.0
    gref = (4.0 / EPS ** 2) * ref["jtr"]
    assert (np.abs(g - gref) <= 1e-4 * gl1).all(), (g, gref, gl1)


def test_autograd_gradient_matches_central_differences(rm):
    """Central differences of the GPU's own E_soft through AlignCost, step
    1e-3 (m / rad) on each se(3) axis, against the gradient AlignCost returns,
    over pixels whose winning triangle, Table I cell and active state are the
    same at all 13 poses (the oracle decides, and flags none of them).

    Step and tolerance follow from the float32 arithmetic of the cost: the
    depth key holds w = 1/z rounded to float32 and z = 1/w is formed in
    float32, so each pixel's residual carries an error of order 2^-23 z and
    its rho one of order 4 |r| 2^-23 z / eps^2 (about 3e-6 at z = 3 m,
    r = 5 cm); summed over the ~2,800 pixels this is E_soft's ~1e-3 offset
    from the FP64 oracle, which the difference quotient divides by 2h.  At
    h = 1e-4 that is ~5e-4 of the gradient's L1 mass (measured), at h = 1e-3
    ~5e-5, inside the 2e-4 allowed here.  (The oracle's own FP64 finite
    differences are checked at h = 1e-4 on the CPU.)"""
    _say("autograd central differences")
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    d, c = O.scan_image(w.scan_depth)
    T = w.poses[0]
    h = 1e-3
    ref = O.align_cost(w.map_mesh, w.cam, T, d, c, eps=EPS)
    t0 = ref["terms"]
    keep = ~flagged_pixels(ref["render"], t0, w.cam, EPS)
    for k in range(6):
        for sgn in (1.0, -1.0):
            e = np.zeros(6); e[k] = sgn * h
            r = O.align_cost(w.map_mesh, w.cam, O.retract(T, e), d, c, eps=EPS)
            tk = r["terms"]
            keep &= (r["render"]["id"] == ref["render"]["id"]) & (tk["cell"] == t0["cell"])
            keep &= (tk["active"] == t0["active"]) & ~flagged_pixels(r["render"], tk, w.cam, EPS)
    assert keep.mean() > 0.8 and t0["active"][keep].sum() > 500
    scan = _tiny_masked_scan(rm, w, keep)
    T0 = _T([T])
    delta = torch.zeros((1, 6), dtype=torch.float64, device=DEV, requires_grad=True)
    rm.AlignCost.apply(delta, T0, dm, scan, EPS).sum().backward()
    g = delta.grad.cpu().numpy()[0]
    fd = np.zeros(6)
    for k in range(6):
        vals = []
        for sgn in (1.0, -1.0):
            dk = torch.zeros((1, 6), dtype=torch.float64, device=DEV)
            dk[0, k] = sgn * h
            vals.append(rm.AlignCost.apply(dk, T0, dm, scan, EPS).item())
        fd[k] = (vals[0] - vals[1]) / (2 * h)
    gl1 = (4.0 / EPS ** 2) * np.abs(t0["r"][keep, None] * t0["J"][keep]).sum(0)
    assert (np.abs(fd - g) <= 2e-4 * gl1).all(), (fd, g, gl1, np.abs(fd - g) / gl1)
    # and the oracle's analytic gradient over the same pixels
    gref = (4.0 / EPS ** 2) * O.reduce_terms(t0, keep)["jtr"]
    assert (np.abs(g - gref) <= 1e-4 * gl1).all(), (g, gref)


def test_graph_replay_matches_eager(rm):
    """An optimizer step (cost + gradient + LM update) captured once and
    replayed several times, with eager work in between, matches running the
    same calls eagerly."""
    _say("graph replay")
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    T0 = _T(w.poses[:8])
    Te = T0.clone()
    eager = []
    out = torch.empty((8, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
    for it in range(3):
        rm.align_cost_grad(dm, scan, Te, 0.3, out=out)
        rm.gn_step(out, Te, 0.01)
        eager.append((out.clone(), Te.clone()))
    Tg = T0.clone()
    outg = torch.empty_like(out)
    rm.align_cost_grad(dm, scan, Tg, 0.3, out=outg)      # sizes the scratch before capture
    torch.cuda.synchronize()
    g = rm.Graph()
    with g:
        rm.align_cost_grad(dm, scan, Tg, 0.3, out=outg)
        rm.gn_step(outg, Tg, 0.01)
    for it in range(3):
        g.replay()
        junk = torch.randn(1000, device=DEV).sum()     # eager work between replays
        torch.cuda.synchronize()
        np.testing.assert_array_equal(outg.cpu().numpy(), eager[it][0].cpu().numpy())
        np.testing.assert_array_equal(Tg.cpu().numpy(), eager[it][1].cpu().numpy())
        del junk


# ------------------------------------------------------------------ alignment drivers

def test_batched_alignment_converges_and_graph_matches(rm):
    """Gauss-Newton with the eps schedule brings 10 cm / 5 deg starts on the
    Kinect-like map (20 smoothed views) to below 2 cm and 0.5 deg within 20
    iterations; replaying the captured graph gives the same poses as eager
    execution, twice in a row."""
    _say("batched alignment")
    from paper_1702_06813_amd import align as A
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    rng = np.random.default_rng(21)
    T0 = _T([S.perturb(w.T_true, rng, 0.10, np.deg2rad(5.0), fixed=True) for _ in range(16)])
    al = A.BatchedAligner(dm, scan, 16, iters=20)
    Te = al.run(T0).clone().cpu().numpy()
    Tg = al.run(T0, use_graph=True).clone()
    Tg2 = al.run(T0, use_graph=True).clone()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Tg.cpu().numpy(), Te)
    np.testing.assert_array_equal(Tg2.cpu().numpy(), Te)
    dt, da = A.pose_errors(Te, w.T_true)
    assert np.median(dt) < 0.02 and dt.max() < 0.04, dt
    assert np.median(da) < np.deg2rad(0.5), np.rad2deg(da)


def test_batched_adam_alignment_converges(rm):
    """Adam on the se(3) gradient (step 4 cm to 2 mm, geometric; moment
    decays 0.5 / 0.9) with the eps schedule brings 10 cm / 5 deg starts on the
    Kinect-like map below 3 cm / 1 deg in 20 iterations (Gauss-Newton reaches
    ~0.7 cm); graph replay equals eager."""
    _say("batched adam alignment")
    from paper_1702_06813_amd import align as A
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    rng = np.random.default_rng(25)
    T0 = _T([S.perturb(w.T_true, rng, 0.10, np.deg2rad(5.0), fixed=True) for _ in range(16)])
    al = A.BatchedAligner(dm, scan, 16, iters=20, method="adam")
    Te = al.run(T0).clone().cpu().numpy()
    Tg = al.run(T0, use_graph=True).clone().cpu().numpy()
    np.testing.assert_array_equal(Tg, Te)
    dt, da = A.pose_errors(Te, w.T_true)
    _say(f"adam: median {np.median(dt) * 100:.2f} cm {np.degrees(np.median(da)):.3f} deg, max {dt.max() * 100:.2f} cm")
    assert np.median(dt) < 0.03 and np.median(da) < np.deg2rad(1.0)


@pytest.mark.slow
def test_trajectory_alignment(rm):
    """48 scans of the looped walk around the office room (320x240, 640x480,
    1280x960 cycling) against the map of its 130 views, meshified by the
    oracle: batches of 32 scans per launch replayed from one graph per batch
    shape give the poses of eager execution bit for bit, and the 10 cm /
    5 deg starts end at a median below 4 cm (the union of 130 noisy views
    leaves a ~2 cm bias)."""
    _say("trajectory alignment (48 scans)")
    from paper_1702_06813_amd import align as A
    from workloads import configs
    tr = configs.trajectory(n_scans=48)
    parts = [O.meshify(d, tr.view_cam, T, tr.stride, tr.z_min, tr.z_max, tr.max_edge, tr.smooth_radius)
             for T, d in zip(tr.views, tr.view_depths)]
    xyz, tri, cls, off = [], [], [], 0
    for v, t, c in parts:
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
    dm = _dev_mesh(rm, (np.concatenate(xyz), np.concatenate(tri).astype(np.int32), np.concatenate(cls)))
    scans = [rm.scan_image(torch.from_numpy(x.depth).to(DEV), tr.z_min, tr.z_max, cam=x.cam) for x in tr.scans]
    T0 = np.stack([x.poses[0] for x in tr.scans])
    truth = np.stack([x.T_true for x in tr.scans])
    ta = A.TrajectoryAligner(dm)
    Tg, launches = ta.run(scans, T0, use_graph=True)
    Te, _ = ta.run(scans, T0, use_graph=False)
    np.testing.assert_array_equal(Tg, Te)
    assert launches == 2 * 20 and len(ta.shapes) == 2
    dt = np.array([A.pose_errors(Tg[j], truth[j])[0][0] for j in range(len(Tg))])
    da = np.degrees(np.array([A.pose_errors(Tg[j], truth[j])[1][0] for j in range(len(Tg))]))
    _say(f"trajectory: median {np.median(dt) * 100:.2f} cm, p90 {np.percentile(dt, 90) * 100:.2f} cm, "
         f"max {dt.max() * 100:.2f} cm; median {np.median(da):.3f} deg")
    assert np.median(dt) < 0.04 and np.median(da) < 1.0


def test_plain_form_reduces_table_cost(rm):
    _say("plain form")
    from paper_1702_06813_amd import align as A
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    rng = np.random.default_rng(22)
    T0 = S.perturb(w.T_true, rng, 0.05, np.deg2rad(2.0), fixed=True)
    e0 = rm.align_cost(dm, scan, _T([T0]), EPS).cpu().numpy()[0, 0]
    T, e, ev = A.plain_align(dm, scan, T0, eps=EPS, budget=300)
    assert ev <= 300 and e < e0
    dt0, _ = A.pose_errors(T0, w.T_true)
    dt, _ = A.pose_errors(T, w.T_true)
    assert dt[0] < dt0[0]


def test_batched_plain_form_matches_plain_form(rm):
    """The paper's optimizer run for several alignments in lockstep (one
    batched launch per round) ends at exactly the poses, costs and evaluation
    counts of running it one alignment at a time."""
    _say("batched plain form")
    from paper_1702_06813_amd import align as A
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    rng = np.random.default_rng(23)
    starts = np.stack([S.perturb(w.T_true, rng, 0.05, np.deg2rad(2.0), fixed=True) for _ in range(3)])
    T, E, ev, launches = A.batched_plain_align(dm, scan, starts, eps=EPS, budget=120)
    for k in range(3):
        Tk, ek, evk = A.plain_align(dm, scan, starts[k], eps=EPS, budget=120)
        np.testing.assert_array_equal(Tk, T[k])
        assert ek == E[k] and evk == ev[k]
    assert launches == ev.max()


def test_plain_form_batched_within_one_alignment(rm):
    """The paper's optimizer for one alignment with its independent points
    (stencil, line-search steps, simplex, Nelder-Mead candidates,
    coordinate-descent probes) evaluated together: exactly the pose, cost
    and evaluation count of the one-point-per-launch form, in under half of
    its launches (under a quarter at the full budget of 700)."""
    _say("plain form batched within one alignment")
    from paper_1702_06813_amd import align as A
    w = workload("kinect")
    dm = _dev_mesh(rm, oracle_map("kinect"))
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    rng = np.random.default_rng(24)
    for k in range(2):
        T0 = S.perturb(w.T_true, rng, 0.05, np.deg2rad(2.0), fixed=True)
        T1, e1, ev1 = A.plain_align(dm, scan, T0, eps=EPS, budget=250)
        T2, e2, ev2, launches = A.plain_align_batched(dm, scan, T0, eps=EPS, budget=250)
        np.testing.assert_array_equal(T1, T2)
        assert e1 == e2 and ev1 == ev2
        assert launches < ev1 / 2, (launches, ev1)
    starts = np.stack([S.perturb(w.T_true, rng, 0.05, np.deg2rad(2.0), fixed=True) for _ in range(3)])
    Ta, Ea, eva, la = A.batched_plain_align(dm, scan, starts, eps=EPS, budget=120)
    Tb, Eb, evb, lb = A.batched_plain_align(dm, scan, starts, eps=EPS, budget=120, speculative=True)
    np.testing.assert_array_equal(Ta, Tb)
    np.testing.assert_array_equal(Ea, Eb)
    np.testing.assert_array_equal(eva, evb)
    assert lb < la


def test_plain_form_visited_points_match_oracle(rm):
    """Every pose the batched plain-form optimizer evaluates on the tiny room
    (speculative points included): the GPU's E_table equals the oracle's
    over the pixels the oracle does not flag at that pose, and differs from
    the oracle's full-frame E_table by at most the flagged pixels."""
    _say("plain form: oracle E_table at visited poses")
    from paper_1702_06813_amd import align as A
    w = workload("tiny")
    dm = _dev_mesh(rm, w.map_mesh)
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
    T0 = w.poses[0]
    T0d = _T([T0])
    seen_T, seen_E = [], []

    def f(xs):
        X = torch.from_numpy(np.stack(xs)).to(DEV)
        Td = rm.se3_retract(T0d.expand(len(xs), 12).contiguous(), X)
        out = rm.align_cost(dm, scan, Td, EPS)
        seen_T.append(Td.cpu().numpy()); seen_E.append(out[:, rm.OUT_E_TABLE].cpu().numpy())
        return seen_E[-1]

    x, fx, ev, nb = A.hybrid_minimize_batched(f, budget=200)
    Ts, Es = np.concatenate(seen_T), np.concatenate(seen_E)
    assert len(Ts) >= ev
    d, c = O.scan_image(w.scan_depth)
    n_flag_total = 0
    for T, e in zip(Ts, Es):
        ref = O.align_cost(w.map_mesh, w.cam, T.reshape(3, 4), d, c, eps=EPS)
        fl = flagged_pixels(ref["render"], ref["terms"], w.cam, EPS)
        n_flag_total += int(fl.sum())
        assert abs(e - ref["e_table"]) <= 2 * fl.sum(), (e, ref["e_table"], fl.sum())
        if fl.any():
            keep = ~fl
            ms = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), cam=w.cam)
            ms.mask = torch.from_numpy(keep.reshape(w.cam.height, w.cam.width).astype(np.uint8)).to(DEV)
            g = rm.align_cost(dm, ms, _T([T]), EPS).cpu().numpy()[0, rm.OUT_E_TABLE]
            assert g == O.reduce_terms(ref["terms"], keep)["e_table"]
        else:
            assert e == ref["e_table"]
    _say(f"{len(Ts)} poses, {n_flag_total} flagged pixels in all")


def test_table_cost_weighted_matches_oracle(rm):
    """Reweighted Table I (rm_table_cost_weighted) on the GPU records of the
    tiny room, over the pixels the oracle does not flag: Table I's printed
    weights give E_TABLE exactly, and arbitrary weights match the oracle's
    per-pixel weighted sum."""
    _say("weighted table cost")
    w = workload("tiny")
    mesh = oracle_map("tiny")
    rng = np.random.default_rng(9)
    poses = [w.T_true, w.poses[0], S.perturb(w.T_true, rng, 0.05, np.deg2rad(3))]
    outs = _cost_case(rm, "tiny", poses, None, grad=False)
    rec = torch.from_numpy(np.stack(outs)).to(DEV)
    e = rm.table_cost_weighted(rec).cpu().numpy()
    np.testing.assert_array_equal(e, np.stack(outs)[:, 0])
    d, c = O.scan_image(w.scan_depth, w.z_min, w.z_max)
    wt = rng.normal(size=9)
    g = rm.table_cost_weighted(rec, wt).cpu().numpy()
    for b, T in enumerate(poses):
        rend = O.render(mesh, w.cam, T)
        terms = O.pixel_terms(rend, mesh[2], d, c, w.cam, EPS)
        keep = ~flagged_pixels(rend, terms, w.cam, EPS)
        ref = O.table_cost_weighted(terms, wt, keep)
        assert abs(g[b] - ref) <= 1e-12 * max(1.0, np.abs(wt).sum() * keep.sum()), (g[b], ref)
