"""GPU parity of the render-accelerated ICP path (Sec. V) against the FP64
oracle, through the C ABI: downsampling (bit-exact), Eq. (2) normals and
vertex normals (to float rounding), the ICP records (counts exact over
unflagged pixels, sums within 1e-4 of their L1 mass), batched rows equal to
single launches, and the sequential depth-image alignment recovering the
motion of a synthetic sequence.  Every input is seeded; every expected value
comes from the oracle or the workload's ground truth."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from workloads import configs, scenes as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = float(np.float32(0.1))


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


def _T(poses):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(poses).reshape(-1, 12))).to(DEV)


def _cam(W, H, f, zn=0.1, zf=16.0):
    return S.Camera(f, f * 1.05, (W - 1) / 2 + 0.3, (H - 1) / 2 - 0.2, W, H, zn, zf)


def test_depth_downsample_bitexact(rm):
    _say("icp downsample")
    rng = np.random.default_rng(20)
    z = rng.uniform(0.0, 10.0, (37, 53)).astype(np.float32)
    for frac, val in ((0.1, 0.0), (0.05, np.nan), (0.05, np.inf), (0.05, -1.0)):
        z[rng.random(z.shape) < frac] = val
    zd = torch.from_numpy(z).to(DEV)
    for f in (1, 2, 3):
        g = rm.depth_downsample(zd, f, 8.0).cpu().numpy()
        ref = O.downsample(z, f, 8.0)
        assert g.shape == ref.shape
        np.testing.assert_array_equal(np.isnan(g), np.isnan(ref))
        np.testing.assert_array_equal(g[np.isfinite(g)], ref[np.isfinite(ref)])


def _room_image(W=160, H=120, f=120.0, seed=21, noise=0.004, dead=0.01):
    scene = S.random_box_room(seed, size=(4.0, 4.0, 2.5), n_boxes=6)
    cam = _cam(W, H, f)
    lo = scene.room_lo
    T = S.look_pose([lo[0] + 1.0, lo[1] + 1.2, 1.4], np.deg2rad(38.0), np.deg2rad(-18.0))
    d = O.downsample(S.range_image(scene, cam, T, seed, noise_rel=noise, dead=dead), 1, 8.0)
    return scene, cam, T, d


def test_depth_normals_match_oracle(rm):
    _say("icp normals")
    _, cam, _, d = _room_image()
    for sigma, radius in ((1.0, 2), (1.7, 4), (0.8, 0)):
        g = rm.depth_normals(torch.from_numpy(d).to(DEV), cam, sigma, radius).cpu().numpy()
        ref = O.depth_normals(d, cam, sigma, radius)
        np.testing.assert_array_equal(np.isnan(g), np.isnan(ref))
        ok = np.isfinite(ref)
        assert ok.mean() > 0.8
        np.testing.assert_allclose(g[ok], ref[ok], rtol=0, atol=2e-6)


def test_vertex_normals_match_oracle(rm):
    _say("icp vertex normals")
    _, cam, T, d = _room_image()
    n = O.depth_normals(d, cam).astype(np.float32)
    for stride in (1, 2, 3):
        g = rm.vertex_normals(torch.from_numpy(n).to(DEV), stride, T).cpu().numpy()
        ref = O.vertex_normals(n, stride, T)
        np.testing.assert_array_equal(np.isnan(g), np.isnan(ref))
        ok = np.isfinite(ref)
        np.testing.assert_allclose(g[ok], ref[ok], rtol=0, atol=1e-6)


def _icp_setup(W=160, H=120):
    scene, cam, T_ref, d = _room_image(W, H)
    mesh = O.meshify(d, cam, T_ref, 1, 0.1, 8.0, 0.1)
    vn = O.vertex_normals(O.depth_normals(d, cam), 1, T_ref).astype(np.float32)
    rng = np.random.default_rng(22)
    T_true = S.perturb(T_ref, rng, 0.03, np.deg2rad(1.5), fixed=True)
    scan_depth = S.range_image(scene, cam, T_true, 23, noise_rel=0.004, dropout=0.02)
    poses = [T_ref, T_true] + [S.perturb(T_true, rng, 0.02, np.deg2rad(1.0)) for _ in range(3)]
    return cam, mesh, vn, scan_depth, poses


def _icp_flags(rend, terms, cam):
    fl = O.flags(rend, cam)
    return fl["near_tie"] | fl["far_tie"] | fl["grazing"] | O.icp_tol_ties(terms, TOL)


def _compare_icp(g, ref, terms, m, tol=1e-4):
    assert g[rm_ICP_N_SCAN] == ref["n_scan"], (g[rm_ICP_N_SCAN], ref["n_scan"])
    assert g[rm_ICP_N_MODEL] == ref["n_model"], (g[rm_ICP_N_MODEL], ref["n_model"])
    assert g[11] == ref["n_assoc"], (g[11], ref["n_assoc"])
    a = terms["assoc"] & m
    e = terms["e"][a]; J = terms["J"][a]
    assert abs(g[0] - ref["cost"]) <= tol * max(np.abs(terms["dz"][a]).sum(), 1e-12), (g[0], ref["cost"])
    assert abs(g[1] - ref["sse"]) <= tol * max((e * e).sum(), 1e-12), (g[1], ref["sse"])
    b_l1 = np.abs(e[:, None] * J).sum(0)
    assert (np.abs(g[18:24] - ref["jtr"]) <= tol * np.maximum(b_l1, 1e-12)).all(), (g[18:24], ref["jtr"])
    assert (np.abs(g[12:18] - ref["grad"]) <= 2 * tol * np.maximum(b_l1, 1e-12)).all()
    H_l1 = np.abs(J[:, :, None] * J[:, None, :]).sum(0)
    iu = np.triu_indices(6)
    assert (np.abs(g[24:45] - ref["jtj"][iu]) <= tol * np.maximum(H_l1[iu], 1e-12)).all()


rm_ICP_N_SCAN, rm_ICP_N_MODEL = 2, 3


def test_icp_cost_grad_matches_oracle(rm):
    """Full frame (several tiles, ragged right and bottom edges): per pose,
    the counts are exact and the sums within 1e-4 of their L1 mass over the
    pixels the oracle does not flag (depth near-ties, far-plane ties, grazing
    views and association decisions within the depth tolerance of tol)."""
    _say("icp cost_grad parity")
    cam, mesh, vn, scan_depth, poses = _icp_setup()
    d, c = O.scan_image(scan_depth, 0.1, 8.0)
    dm = rm.Mesh.from_arrays(*mesh, device=DEV).prepare()
    vnd = torch.from_numpy(vn).to(DEV)
    scan = rm.scan_image(torch.from_numpy(scan_depth).to(DEV), 0.1, 8.0, cam=cam)
    for b, T in enumerate(poses):
        rend = O.render(mesh, cam, T)
        terms = O.icp_terms(rend, mesh, vn, d, c, cam, T, TOL)
        keep = ~_icp_flags(rend, terms, cam)
        ref = O.icp_reduce(terms, keep)
        mask = np.zeros(cam.width * cam.height, np.uint8)
        mask[rend["pixels"][keep]] = 1
        scan.mask = torch.from_numpy(mask.reshape(cam.height, cam.width)).to(DEV)
        g = rm.icp_cost_grad(dm, scan, _T([T]), vnd, TOL).cpu().numpy()[0]
        _compare_icp(g, ref, terms, keep)
        assert keep.mean() > 0.95 and ref["n_assoc"] > 1000
        assert g[45] > 0                          # clusters survived the cull


def test_icp_batched_rows_equal_single_launches(rm):
    _say("icp batched rows")
    cam, mesh, vn, scan_depth, poses = _icp_setup()
    dm = rm.Mesh.from_arrays(*mesh, device=DEV).prepare()
    vnd = torch.from_numpy(vn).to(DEV)
    scan = rm.scan_image(torch.from_numpy(scan_depth).to(DEV), 0.1, 8.0, cam=cam)
    half = rm.scan_image(torch.from_numpy(np.ascontiguousarray(scan_depth[::2, ::2])).to(DEV), 0.1, 8.0,
                         cam=rm.downsample_camera(cam, 2))
    T = _T(poses + poses[:3])
    allr = rm.icp_cost_grad(dm, [scan, half], T, vnd, TOL, poses_per_scan=[len(poses), 3]).cpu().numpy()
    for i in range(len(poses)):
        one = rm.icp_cost_grad(dm, scan, T[i:i + 1].contiguous(), vnd, TOL).cpu().numpy()
        np.testing.assert_array_equal(one[0], allr[i])
    for i in range(3):
        one = rm.icp_cost_grad(dm, half, T[len(poses) + i:len(poses) + i + 1].contiguous(), vnd, TOL).cpu().numpy()
        np.testing.assert_array_equal(one[0], allr[len(poses) + i])


def test_icp_rejects_bad_arguments(rm):
    cam, mesh, vn, scan_depth, poses = _icp_setup(64, 48)
    dm = rm.Mesh.from_arrays(*mesh, device=DEV).prepare()
    scan = rm.scan_image(torch.from_numpy(scan_depth).to(DEV), 0.1, 8.0, cam=cam)
    with pytest.raises(rm.RenderMapError):
        rm.icp_cost_grad(dm, scan, _T(poses[:1]), torch.from_numpy(vn).to(DEV), -1.0)
    with pytest.raises(rm.RenderMapError):
        rm.depth_normals(torch.from_numpy(scan_depth).to(DEV), cam, 1.0, 99)
    with pytest.raises(ValueError):
        rm.icp_cost_grad(dm, scan, _T(poses[:1]), torch.from_numpy(vn[:-1]).to(DEV), TOL)


def test_sequential_depth_alignment_recovers_motion(rm):
    """Sec. V-B on 9 Kinect-like frames (8 pairs solved in the same launches,
    each model at its own offset): every relative pose is recovered to 5 mm
    and 0.25 degrees from the identity start (motion 3.5 cm / 1.5 deg)."""
    _say("icp sequential alignment")
    from paper_1702_06813_amd import align
    seq = configs.odometry(n_frames=9)
    depths = [torch.from_numpy(d).to(DEV) for d in seq.depths]
    rel, out = align.sequential_depth_alignment(depths, seq.cam, iters=12)
    assert rel.shape == (8, 3, 4)
    for k in range(8):
        T0 = np.vstack([seq.poses[k], [0, 0, 0, 1]])
        T1 = np.vstack([seq.poses[k + 1], [0, 0, 0, 1]])
        truth = (np.linalg.inv(T0) @ T1)[:3]
        dt, ang = align.pose_errors(rel[k][None], truth)
        _say(f"  pair {k}: {dt[0] * 1e3:.2f} mm {np.rad2deg(ang[0]):.3f} deg")
        assert dt[0] < 5e-3 and np.rad2deg(ang[0]) < 0.25, (k, dt[0], np.rad2deg(ang[0]))
    o = out.cpu().numpy()
    assert (o[:, 11] > 10000).all()               # associated pixels per pair at 320x240


@pytest.mark.slow
def test_icp_full_batch_sampled(rm):
    """The benchmark's launch: 32 consecutive pairs of the 33-frame sequence
    at 320x240, every pair's model (built by the oracle) at its own offset,
    4.5M triangles, 32 scans in one launch.  Three pairs are checked on 1500
    sampled pixels each (scan masks) against the oracle rendering the whole
    mesh; all 32 rows of the launch equal single-scan launches."""
    _say("icp full batch (32 pairs, 4.5M triangles)")
    from paper_1702_06813_amd import align
    seq = configs.odometry(n_frames=33)
    cam2 = O.downsample_camera(seq.cam, 2)
    ds = [O.downsample(d, 2, 8.0) for d in seq.depths]
    xyz, tri, cls, vns, offs, off = [], [], [], [], [], 0
    for k in range(32):
        To = np.zeros((3, 4)); To[:, :3] = np.eye(3); To[:, 3] = align._pair_offset(k, 50.0)
        v, t, c = O.meshify(ds[k], cam2, To, 1, 0.1, 8.0, 0.1)
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
        vns.append(O.vertex_normals(O.depth_normals(ds[k], cam2), 1, To).astype(np.float32))
        offs.append(To)
    mesh = (np.concatenate(xyz), np.concatenate(tri).astype(np.int32), np.concatenate(cls))
    vn = np.concatenate(vns)
    assert mesh[1].shape[0] > 4_000_000
    dm = rm.Mesh.from_arrays(*mesh, device=DEV).prepare()
    vnd = torch.from_numpy(vn).to(DEV)
    scans = [rm.scan_image(torch.from_numpy(ds[k + 1]).to(DEV), 0.1, 8.0, cam=cam2) for k in range(32)]
    rng = np.random.default_rng(24)
    poses = [S.perturb(offs[k], rng, 0.01, np.deg2rad(0.5)) for k in range(32)]
    T = _T(poses)
    allr = rm.icp_cost_grad(dm, scans, T, vnd, TOL, poses_per_scan=[1] * 32).cpu().numpy()
    for k in (0, 13, 31):
        one = rm.icp_cost_grad(dm, scans[k], T[k:k + 1].contiguous(), vnd, TOL).cpu().numpy()
        np.testing.assert_array_equal(one[0], allr[k])
    for k in (2, 17, 30):
        d, c = O.scan_image(ds[k + 1], 0.1, 8.0)
        pix = np.sort(rng.choice(cam2.width * cam2.height, 1500, replace=False)).astype(np.int64)
        rend = O.render(mesh, cam2, poses[k], pix)
        terms = O.icp_terms(rend, mesh, vn, d, c, cam2, poses[k], TOL)
        keep = ~_icp_flags(rend, terms, cam2)
        ref = O.icp_reduce(terms, keep)
        mask = np.zeros(cam2.width * cam2.height, np.uint8)
        mask[pix[keep]] = 1
        scans[k].mask = torch.from_numpy(mask.reshape(cam2.height, cam2.width)).to(DEV)
        g = rm.icp_cost_grad(dm, scans, T, vnd, TOL, poses_per_scan=[1] * 32).cpu().numpy()[k]
        scans[k].mask = None
        _compare_icp(g, ref, terms, keep)
        assert keep.mean() > 0.95 and ref["n_assoc"] > 500


def test_icp_empty_and_degenerate(rm):
    """Degenerate inputs of the ICP path: an all-invalid scan associates
    nothing; a pose looking away from the model sees no model pixels and its
    LM step leaves the pose unchanged (H = 0 is not positive definite); the
    normals of tiny and all-invalid images are all NaN, as in the oracle;
    zero poses is a no-op."""
    _say("icp degenerate")
    cam, mesh, vn, scan_depth, poses = _icp_setup(64, 48)
    dm = rm.Mesh.from_arrays(*mesh, device=DEV).prepare()
    vnd = torch.from_numpy(vn).to(DEV)
    dead = rm.scan_image(torch.full((48, 64), float("nan"), device=DEV), 0.1, 8.0, cam=cam)
    g = rm.icp_cost_grad(dm, dead, _T(poses[:1]), vnd, TOL).cpu().numpy()[0]
    assert g[2] == 0 and g[3] == 0 and g[11] == 0 and not g[:2].any() and not g[12:45].any()
    away = poses[0].copy()
    away[:, :3] = away[:, :3] @ np.diag([-1.0, 1.0, -1.0])      # turned half round about its y axis
    scan = rm.scan_image(torch.from_numpy(scan_depth).to(DEV), 0.1, 8.0, cam=cam)
    T = _T([away])
    out = rm.icp_cost_grad(dm, scan, T, vnd, TOL)
    o = out.cpu().numpy()[0]
    rend = O.render(mesh, cam, away)
    d, c = O.scan_image(scan_depth, 0.1, 8.0)
    ref = O.icp_reduce(O.icp_terms(rend, mesh, vn, d, c, cam, away, TOL))
    assert o[2] == ref["n_scan"] and o[3] == ref["n_model"] == 0 and o[11] == 0
    T0 = T.clone()
    rm.gn_step(out, T, 1e-6)
    assert torch.equal(T, T0)
    for img in (np.full((2, 3), 2.0, np.float32), np.full((9, 11), np.nan, np.float32)):
        cam_i = S.Camera(50.0, 50.0, (img.shape[1] - 1) / 2, (img.shape[0] - 1) / 2, img.shape[1], img.shape[0],
                         0.1, 16.0)
        n = rm.depth_normals(torch.from_numpy(img).to(DEV), cam_i).cpu().numpy()
        assert np.isnan(n).all() and np.isnan(O.depth_normals(img, cam_i)).all()
    empty = rm.icp_cost_grad(dm, scan, torch.zeros((0, 12), dtype=torch.float64, device=DEV), vnd, TOL,
                             poses_per_scan=[0])
    assert tuple(empty.shape) == (0, rm.OUT_STRIDE)
