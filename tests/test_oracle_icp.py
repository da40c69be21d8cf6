"""Pins of the oracle's render-accelerated point-to-plane ICP (Sec. V):
Gaussian smoothing against linear ramps and impulses, Eq. (2) normals against
a fronto-parallel plane, tangent orthogonality and a tilted plane at the
principal point, vertex-normal rotation, zero residual at the true pose, the
Jacobian against finite differences of its residual, and Gauss-Newton
convergence of the full render / associate / solve loop.  CPU only."""
import numpy as np
import pytest

from workloads import scenes as S


def _cam(W, H, f, zn=0.1, zf=16.0):
    return S.Camera(f, f, (W - 1) / 2, (H - 1) / 2, W, H, zn, zf)


def test_smoothing_keeps_ramps_renormalizes_holes_and_spreads_impulses(oracle_mod):
    O = oracle_mod
    H, W, R = 20, 24, 2
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    ramp = 2.0 + 0.01 * u - 0.02 * v
    sm = O.smooth_depth(ramp, 1.3, R)
    np.testing.assert_allclose(sm[R:-R, R:-R], ramp[R:-R, R:-R], rtol=0, atol=1e-13)
    # a hole in a constant image: the renormalized weights give the constant back
    c = np.full((H, W), 3.25)
    c[7, 9] = np.nan
    sc = O.smooth_depth(c, 1.0, R)
    assert np.isnan(sc[7, 9])
    np.testing.assert_allclose(sc[np.isfinite(c)], 3.25, rtol=1e-15)
    # an impulse on a constant background spreads as the outer product of the 1-D weights
    im = np.ones((H, W))
    im[10, 12] += 1.0
    w = O.gaussian_weights(1.0, R)
    np.testing.assert_allclose(w.sum(), 1.0, rtol=1e-15)
    np.testing.assert_allclose(w, w[::-1], rtol=0, atol=0)
    si = O.smooth_depth(im, 1.0, R)
    np.testing.assert_allclose(si[8:13, 10:15] - 1.0, np.outer(w, w), rtol=1e-12)


def test_normals_fronto_parallel_plane(oracle_mod):
    O = oracle_mod
    cam = _cam(32, 24, 30.0)
    N = O.depth_normals(np.full((24, 32), 2.5, np.float32), cam)
    inner = N[1:-1, 1:-1].reshape(-1, 3)
    np.testing.assert_allclose(inner, np.tile([0.0, 0.0, -1.0], (inner.shape[0], 1)), atol=1e-12)
    assert np.isnan(N[0]).all() and np.isnan(N[-1]).all() and np.isnan(N[:, 0]).all()


def test_normals_orthogonal_to_both_tangents_and_face_the_camera(oracle_mod):
    """N is perpendicular to (dx, 0, dz_x) and (0, dy, dz_y) of the smoothed
    image (a transposed or mis-signed cross product fails this)."""
    O = oracle_mod
    cam = _cam(40, 30, 35.0)
    rng = np.random.default_rng(3)
    v, u = np.mgrid[0:30, 0:40].astype(np.float64)
    z = 2.0 + 0.3 * np.sin(u / 7.0) + 0.2 * np.cos(v / 5.0) + 0.01 * rng.standard_normal(u.shape)
    N = O.depth_normals(z, cam, 1.0, 2)
    zs = O.smooth_depth(z, 1.0, 2)
    c = zs[1:-1, 1:-1]
    tx = np.stack([2 * c / cam.fx, np.zeros_like(c), zs[1:-1, 2:] - zs[1:-1, :-2]], -1)
    ty = np.stack([np.zeros_like(c), 2 * c / cam.fy, zs[2:, 1:-1] - zs[:-2, 1:-1]], -1)
    n = N[1:-1, 1:-1]
    np.testing.assert_allclose((n * tx).sum(-1), 0.0, atol=1e-14)
    np.testing.assert_allclose((n * ty).sum(-1), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(n, axis=-1), 1.0, rtol=1e-14)
    assert (n[..., 2] < 0).all()


def test_normals_match_a_tilted_plane_at_the_principal_point(oracle_mod):
    """At the principal point the image-plane tangents of Eq. (2) are the
    surface tangents, so the normal of a tilted plane is recovered there
    (to the central-difference error of the projected depth)."""
    O = oracle_mod
    cam = S.Camera(40.0, 55.0, 20.0, 15.0, 41, 31, 0.1, 16.0)   # fx != fy; principal point at pixel (20, 15)
    n_true = np.array([0.3, -0.2, -1.0]); n_true /= np.linalg.norm(n_true)
    c = -2.0                                     # plane n . X = c, in front of the camera
    r = O.rays(cam, np.arange(41 * 31)).reshape(31, 41, 3)
    z = c / (r @ n_true)
    N = O.depth_normals(z, cam, 1.0, 2)
    np.testing.assert_allclose(N[15, 20], n_true, atol=2e-3)
    # away from the principal point the height-field normal departs from the plane's
    assert np.abs(N[2, 3] - n_true).max() > 1e-2


def test_vertex_normals_take_node_pixels_and_rotate(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(4)
    N = rng.standard_normal((9, 10, 3))
    T = np.zeros((3, 4))
    ang = 0.7
    T[:, :3] = [[np.cos(ang), 0, np.sin(ang)], [0, 1, 0], [-np.sin(ang), 0, np.cos(ang)]]
    T[:, 3] = [1.0, 2.0, 3.0]
    vn = O.vertex_normals(N, 3, T)
    assert vn.shape == (3 * 4, 3)
    np.testing.assert_allclose(vn[1 * 4 + 2], T[:, :3] @ N[3, 6], rtol=1e-14)


def _room_pair(O, W=80, H=60, f=60.0, seed=7):
    scene = S.random_box_room(seed, size=(4.0, 4.0, 2.5), n_boxes=6)
    cam = _cam(W, H, f)
    lo, hi = scene.room_lo, scene.room_hi
    T_ref = S.look_pose([lo[0] + 1.0, lo[1] + 1.0, 1.4], np.deg2rad(40.0), np.deg2rad(-15.0))
    ref = O.downsample(S.range_image(scene, cam, T_ref, 0, noise_rel=0.0), 1, 8.0)
    mesh = O.meshify(ref, cam, T_ref, 1, 0.1, 8.0, 0.1)
    vn = O.vertex_normals(O.depth_normals(ref, cam), 1, T_ref)
    return scene, cam, T_ref, mesh, vn


def test_icp_residual_vanishes_at_the_true_pose(oracle_mod):
    O = oracle_mod
    scene, cam, T_ref, mesh, vn = _room_pair(O)
    rend = O.render(mesh, cam, T_ref)
    zr = np.where(rend["id"] >= 0, rend["z"], np.nan).reshape(cam.height, cam.width)
    d, c = O.scan_image(np.where(np.isfinite(zr), zr, 0.0).astype(np.float32), 0.1, 8.0)
    out = O.icp_step(mesh, vn, cam, T_ref, d, c, 0.05)
    t = out["terms"]
    assert out["n_assoc"] > 0.5 * cam.width * cam.height
    # e = (z1 - zM) (n . r) with z1 = fl32(zM): only the float32 rounding of the scan remains
    assert np.abs(t["e"]).max() < 1e-6
    assert np.abs(out["jtr"]).max() < 1e-6 * out["n_assoc"]


def test_icp_jacobian_matches_finite_differences_of_its_residual(oracle_mod):
    """J = [n ; P_1 x n] is the derivative of e = n . (exp(delta) P_1 - P_M)
    with the correspondence (P_M, n) held, as point-to-plane ICP linearizes."""
    O = oracle_mod
    scene, cam, T_ref, mesh, vn = _room_pair(O)
    T = O.retract(T_ref, np.array([0.01, -0.005, 0.008, 0.004, -0.006, 0.003]))
    d, c = O.scan_image(S.range_image(scene, cam, T, 0, noise_rel=0.0), 0.1, 8.0)
    out = O.icp_step(mesh, vn, cam, T, d, c, 0.1)
    t = out["terms"]
    idx = np.flatnonzero(t["assoc"])[::7][:60]
    ray = O.rays(cam, out["render"]["pixels"][idx])
    P1 = t["z1"][idx, None] * ray
    PM = t["zM"][idx, None] * ray
    n = t["n"][idx]
    h = 1e-6
    for k in range(6):
        e = np.zeros(6); e[k] = h
        Tp, Tm = O.se3_exp(e), O.se3_exp(-e)
        fp = ((P1 @ Tp[:3, :3].T + Tp[:3, 3] - PM) * n).sum(-1)
        fm = ((P1 @ Tm[:3, :3].T + Tm[:3, 3] - PM) * n).sum(-1)
        np.testing.assert_allclose((fp - fm) / (2 * h), t["J"][idx, k], rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(((P1 - PM) * n).sum(-1), t["e"][idx], rtol=1e-12, atol=1e-15)


def test_icp_gauss_newton_recovers_the_motion(oracle_mod):
    """Noise-free frame pair in a box room, 3 cm / 2 deg apart: the render /
    associate / solve loop from the reference pose reaches the true pose."""
    O = oracle_mod
    scene, cam, T_ref, mesh, vn = _room_pair(O)
    rng = np.random.default_rng(11)
    T_true = S.perturb(T_ref, rng, 0.03, np.deg2rad(2.0), fixed=True)
    d, c = O.scan_image(S.range_image(scene, cam, T_true, 0, noise_rel=0.0), 0.1, 8.0)
    T = T_ref.copy()
    for it in range(15):
        out = O.icp_step(mesh, vn, cam, T, d, c, 0.1)
        T = O.retract(T, O.gn_step(out, 1e-6))
    dt = np.linalg.norm(T[:, 3] - T_true[:, 3])
    ang = np.arccos(np.clip((np.trace(T[:, :3].T @ T_true[:, :3]) - 1) / 2, -1, 1))
    assert dt < 1e-3 and np.rad2deg(ang) < 0.05, (dt, np.rad2deg(ang))


def test_downsample_keeps_every_other_pixel_and_filters_far(oracle_mod):
    O = oracle_mod
    d = np.arange(48, dtype=np.float32).reshape(6, 8) * 0.25
    d[0, 2] = 0.0
    d[2, 4] = np.nan
    out = O.downsample(d, 2, 8.0)
    assert out.shape == (3, 4)
    ref = d[::2, ::2].copy()
    ref[(ref <= 0) | (ref > 8.0) | ~np.isfinite(ref)] = np.nan
    np.testing.assert_array_equal(np.isnan(out), np.isnan(ref))
    np.testing.assert_array_equal(out[np.isfinite(out)], ref[np.isfinite(ref)])
    cam2 = O.downsample_camera(_cam(8, 6, 10.0), 2)
    assert (cam2.width, cam2.height) == (4, 3) and cam2.fx == 5.0 and cam2.cx == 3.5 / 2
