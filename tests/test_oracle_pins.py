"""Pins of the FP64 oracle against facts fixed by the paper and by geometry:
closed-form depths, watertightness, fill-rule ownership, Table I as printed,
zero cost at the true pose, finite differences, Gauss-Newton convergence,
SE(3) against scipy, and meshification counts.  CPU only."""
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from workloads import configs, scenes as S

GOLDEN = Path(__file__).resolve().parent / "golden"


def _cam(W, H, f, cx=None, cy=None, zn=0.1, zf=16.0):
    return S.Camera(f, f, (W - 1) / 2 if cx is None else cx, (H - 1) / 2 if cy is None else cy, W, H, zn, zf)


def _identity():
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    return T


# ---------------------------------------------------------------- depth pins

def test_plane_closed_form(oracle_mod):
    """A dyadic tilted plane z = 2 + x/4 + y/8 seen from the identity pose:
    z(u,v) = 2 / (1 - r_x/4 - r_y/8) for every pixel, in both coverage modes."""
    O = oracle_mod
    mesh = S.plane_mesh(n_per_side=8, extent=4.0, z0=2.0, slope=(0.25, 0.125))
    cam = _cam(64, 48, 40.0)
    r = O.rays(cam, np.arange(64 * 48))
    z_cf = 2.0 / (1.0 - 0.25 * r[:, 0] - 0.125 * r[:, 1])
    for mode in ("contract", "exact"):
        out = O.render(mesh, cam, _identity(), mode=mode)
        assert (out["id"] >= 0).all()
        np.testing.assert_allclose(out["z"], z_cf, rtol=1e-12)


@pytest.mark.parametrize("k", range(4))
def test_box_room_closed_form(oracle_mod, k):
    """Triangulated box room: exact-mode depth equals the analytic ray/box
    depth to 1e-12 everywhere; contract mode has no empty pixel (closed room)
    and agrees with exact mode except at pixel centres within a snap step of a
    triangle edge."""
    O = oracle_mod
    rng = np.random.default_rng(10 + k)
    scene = S.random_box_room(k, (4.0, 4.0, 2.5), 8)
    mesh = S.triangulate_scene(scene, 0.25)
    T = S.look_pose(np.array([rng.uniform(1, 3), rng.uniform(1, 3), rng.uniform(0.9, 1.8)]),
                    rng.uniform(0, 2 * np.pi), rng.uniform(-0.6, 0.6), rng.uniform(-0.4, 0.4))
    cam = _cam(96, 72, 70.0)
    z_an = S.analytic_depth(scene, cam, T).ravel()
    ex = O.render(mesh, cam, T, mode="exact")
    np.testing.assert_allclose(ex["z"], z_an, rtol=1e-12)
    ct = O.render(mesh, cam, T, mode="contract")
    assert (ct["id"] >= 0).all(), "closed room must have no empty pixel"
    assert (ct["ncov"] >= 1).all()
    rel = np.abs(ct["z"] - z_an) / z_an
    assert np.mean(rel > 1e-9) < 0.02
    assert np.max(rel) < 2e-2


def test_watertight_plane_grid_single_coverage(oracle_mod):
    """A planar grid whose vertices project exactly onto pixel centres covers
    every pixel centre inside it exactly once (top-left rule on shared edges)."""
    O = oracle_mod
    cam = S.Camera(8.0, 8.0, 0.0, 0.0, 16, 16, 0.1, 16.0)
    # fronto-parallel plane z = 1: vertex x = k/8 projects to u = k exactly
    k = np.arange(0, 17, 2, dtype=np.float64) / 8.0
    xx, yy = np.meshgrid(k, k, indexing="ij")
    xyz = np.stack([xx, yy, np.ones_like(xx)], -1).reshape(-1, 3).astype(np.float32)
    n = len(k)
    idx = np.arange(n * n).reshape(n, n)
    q00, q01, q10, q11 = idx[:-1, :-1].ravel(), idx[:-1, 1:].ravel(), idx[1:, :-1].ravel(), idx[1:, 1:].ravel()
    tri = np.concatenate([np.stack([q00, q01, q11], 1), np.stack([q00, q11, q10], 1)]).astype(np.int32)
    out = O.render((xyz, tri, np.zeros(len(tri), np.uint8)), cam, _identity())
    ncov = out["ncov"].reshape(16, 16)
    # the grid spans pixel centres [0, 16] in u and v; the right and bottom
    # outer edges are not top-left, so columns/rows 16 are outside the image anyway
    assert (ncov == 1).all()


def test_top_left_ownership(oracle_mod):
    """Hand-derived ownership of pixel centres on triangle edges (y down):
    a horizontal edge with the interior below it (top edge) and an edge with
    the interior to its right (left edge) own their pixel centres; bottom and
    right edges do not."""
    O = oracle_mod
    cam = S.Camera(8.0, 8.0, 0.0, 0.0, 12, 12, 0.1, 16.0)

    def cover(pts):
        xyz = np.array([[x / 8.0, y / 8.0, 1.0] for x, y in pts], np.float32)
        out = O.render((xyz, np.array([[0, 1, 2]], np.int32), np.zeros(1, np.uint8)), cam, _identity())
        return out["ncov"].reshape(12, 12)

    # right triangle with a top edge on row 2 (x 2..8) and a left edge on column 2 (y 2..8)
    c = cover([(2, 2), (8, 2), (2, 8)])
    assert c[2, 2:8].all() and c[2, 8] == 0          # top edge owned, far vertex (8,2) is on the hypotenuse
    assert c[2:8, 2].all()                           # left edge owned
    # the mirrored triangle has a bottom edge on row 8 and a right edge on column 8
    c2 = cover([(8, 8), (2, 8), (8, 2)])
    assert not c2[8, :].any() and not c2[:, 8].any()
    # together they tile the square [2,8]^2 with no overlap: the shared
    # diagonal x + y = 10 is owned by exactly one of them
    both = c + c2
    assert both.max() == 1
    assert (both[2:8, 2:8] == 1).all()
    # orientation does not matter
    assert (cover([(2, 2), (2, 8), (8, 2)]) == c).all()


def test_orientation_flip_invariance(oracle_mod):
    O = oracle_mod
    w = configs.tiny()
    xyz, tri, cls = w.map_mesh
    a = O.render((xyz, tri, cls), w.cam, w.poses[0])
    b = O.render((xyz, tri[:, ::-1].copy(), cls), w.cam, w.poses[0])
    assert (a["id"] == b["id"]).all()
    np.testing.assert_allclose(a["z"], b["z"], rtol=1e-14)   # plane from permuted vertices: rounding only


def test_contract_vs_exact_mismatch_rate(oracle_mod):
    """Snapping to 1/256 px only changes ownership of pixel centres very close
    to an edge."""
    O = oracle_mod
    w = configs.tiny()
    for T in (w.T_true, w.poses[0]):
        a = O.render(w.map_mesh, w.cam, T, mode="contract")
        b = O.render(w.map_mesh, w.cam, T, mode="exact")
        assert np.mean(a["id"] != b["id"]) < 0.01


def test_near_plane_clip_keeps_front_part(oracle_mod):
    """A floor triangle that passes behind the camera is clipped at z_near:
    pixels that see the floor in front of the camera keep the closed-form
    depth, and the clip moves no pixel off the floor."""
    O = oracle_mod
    cam = _cam(64, 48, 40.0, zn=0.1)
    # floor y = +1 (camera frame, y down) spanning z in [-5, 20]
    xyz = np.array([[-30, 1, -5], [30, 1, -5], [0, 1, 20]], np.float32)
    mesh = (xyz, np.array([[0, 1, 2]], np.int32), np.zeros(1, np.uint8))
    pix = np.arange(64 * 48)
    r = O.rays(cam, pix)
    a = O.render(mesh, cam, _identity(), mode="contract")
    b = O.render(mesh, cam, _identity(), mode="exact")
    z_cf = 1.0 / r[:, 1]
    hit = a["id"] >= 0
    np.testing.assert_allclose(a["z"][hit], z_cf[hit], rtol=1e-12)
    assert np.mean(hit != (b["id"] >= 0)) < 0.02
    assert hit.sum() > 0


# ---------------------------------------------------------------- Table I

def _parse_table():
    rows = {}
    for line in (GOLDEN / "table1.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        m, s, rule = line.split(None, 2)
        rows[(m, s)] = rule.strip()
    return rows


def _eval_rule(rule, dz, eps):
    if rule in ("ignore", "N/A"):
        return 0
    for part in rule.split(";"):
        val, cond = part.strip().split(" if ")
        lhs, op, rhs = cond.split()
        x = abs(dz) if lhs == "|dz|" else dz
        y = eps if rhs == "eps" else float(rhs)
        ok = {"<=": x <= y, ">": x > y, "<": x < y, ">=": x >= y}[op]
        if ok:
            return int(val)
    raise AssertionError(rule)


def test_table1_matches_paper_exhaustively(oracle_mod):
    O = oracle_mod
    eps = 0.1
    code = {"FO": O.FO, "FU": O.FU, "UO": O.UO, "NaN": O.NONE}
    table = _parse_table()
    assert len(table) == 16
    for (m, s), rule in table.items():
        for k in (-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0, -1e-9, 1e-9):
            dz = k * eps
            got, cell = O.table1(np.array([code[m]]), np.array([code[s]]), np.array([dz]), eps)
            assert got[0] == _eval_rule(rule, dz, eps), (m, s, dz)
            assert 0 <= cell[0] < 9


def test_table1_counts_invariants(oracle_mod):
    O = oracle_mod
    w = configs.tiny()
    d, c = O.scan_image(w.scan_depth)
    out = O.align_cost(w.map_mesh, w.cam, w.poses[0], d, c)
    cnt = out["counts"]
    assert cnt.sum() == w.cam.width * w.cam.height
    assert out["e_table"] == (cnt[1] + cnt[3] + cnt[5]) - (cnt[0] + cnt[2] + cnt[4])


def test_soft_cost_agrees_with_table_outside_band(oracle_mod):
    """rho = Table I value wherever |r| >= eps, and rho = -1 on reward cells
    with r = 0 (E_soft is continuous and bounded in [-1, 1])."""
    O = oracle_mod
    eps = 0.1
    rng = np.random.default_rng(3)
    n = 4000
    c_r = rng.integers(0, 4, n); c_s = rng.choice([0, 1, 3], n)
    dz = rng.uniform(-0.4, 0.4, n)
    s, _ = O.table1(c_r, c_s, dz, eps)
    r, scored, _ = O.residual(c_r, c_s, dz)
    rho = np.where(scored, 2 * np.minimum(r * r / eps ** 2, 1) - 1, 0)
    far = scored & (np.abs(r) >= eps)
    assert (rho[far] == s[far]).all()
    zero_reward = scored & (r == 0) & (s == -1)
    assert (rho[zero_reward] == -1).all()
    assert (np.abs(rho) <= 1).all()


# ---------------------------------------------------------------- cost pins

def test_zero_cost_at_true_pose(oracle_mod):
    """Noiseless scan of the tiny room rendered analytically at T*: every
    pixel is FO/FO with r ~ 0, so E_table = E_soft = -N and the gradient is
    zero relative to the L1 mass of the per-pixel gradient terms."""
    O = oracle_mod
    w = configs.tiny()
    depth = S.range_image(w.scene, w.cam, w.T_true, 0, noise_rel=0.0)
    d, c = O.scan_image(depth)
    out = O.align_cost(w.map_mesh, w.cam, w.T_true, d, c)
    t = out["terms"]
    N = w.cam.width * w.cam.height
    assert out["counts"][0] == N
    assert out["e_table"] == -N
    assert np.max(np.abs(t["r"])) < 2e-6      # float32 scan depths
    assert abs(out["e_soft"] + N) < 1e-6 * N
    # residuals are float32 rounding of the scan only: J^T r is bounded by that
    # rounding times sum |J|, and tiny next to its value 1 cm away from T*
    assert (np.abs(out["jtr"]) <= 2e-6 * np.abs(t["J"]).sum(0)).all()
    T_off = w.T_true.copy(); T_off[:, 3] += np.array([0.01, -0.006, 0.004])
    off = O.align_cost(w.map_mesh, w.cam, T_off, d, c)
    assert np.linalg.norm(out["jtr"]) < 1e-3 * np.linalg.norm(off["jtr"])


def test_jacobian_matches_finite_differences(oracle_mod):
    """J_p is the derivative of the residual e_p (the scan point's signed
    distance from the plane of the triangle the pixel sees) under a right
    perturbation T exp(delta): central differences with step 1e-4 agree to
    1e-6 on pixels whose winning triangle does not change."""
    O = oracle_mod
    w = configs.tiny()
    rng = np.random.default_rng(5)
    pix = rng.choice(w.cam.width * w.cam.height, 400, replace=False)
    d, c = O.scan_image(w.scan_depth)
    fd, stable, t = O.fd_jacobian(w.map_mesh, w.cam, w.poses[0], pix, d, c, h=1e-4)
    m = stable & t["active"]
    assert m.sum() > 300
    J = t["J"]
    err = np.abs(fd[m] - J[m]).max(0) / np.abs(J[m]).max(0)
    assert (err < 1e-6).all(), err
    # e_p is the point-to-plane distance: |e_p| = |dz| |n^.ray| <= |dz| |ray|,
    # equal to |dz| on the optical axis of a plane facing the camera
    assert (np.abs(t["dz"][m] * t["g"][m]) <= np.abs(t["dz"][m]) * t["ray_norm"][m] + 1e-15).all()


def test_residual_is_distance_between_parallel_planes(oracle_mod):
    """Map: the tilted plane z = 2 + x/4 + y/8.  Scan: the same plane moved
    3 cm towards the camera along its normal.  Every scan point then lies
    exactly 3 cm from the map plane on the camera side, so r_p = +0.03 at
    every pixel, while dz varies across the image with the ray's obliquity."""
    O = oracle_mod
    cam = _cam(64, 48, 40.0)
    plane = S.plane_mesh(16, 8.0)
    n = np.array([-0.25, -0.125, 1.0]); n /= np.linalg.norm(n)
    delta = 0.03
    c = n @ np.array([0.0, 0.0, 2.0]) - delta
    u, v = np.meshgrid(np.arange(64.0), np.arange(48.0))
    ray = np.stack([(u - cam.cx) / cam.fx, (v - cam.cy) / cam.fy, np.ones_like(u)], -1)
    d_s = (c / (ray @ n)).astype(np.float32)
    d, cl = O.scan_image(d_s)
    out = O.align_cost(plane, cam, _identity(), d, cl, eps=0.1)
    t = out["terms"]
    assert out["counts"][0] == 64 * 48
    np.testing.assert_allclose(t["r"], delta, atol=1e-6)
    assert np.ptp(t["dz"]) > 0.005           # dz itself is not constant
    assert out["n_active"] == 64 * 48


def _corner_setup():
    scene = S.Scene(np.zeros(3), np.array([4.0, 4.0, 2.5]), np.zeros((0, 2, 3)))
    mesh = S.triangulate_scene(scene, 0.25)
    T = S.look_pose(np.array([2.6, 2.6, 1.3]), np.deg2rad(225.0) + np.pi, np.deg2rad(-25.0))
    return scene, mesh, T


def test_hessian_rank_plane_vs_corner(oracle_mod):
    O = oracle_mod
    scene, mesh, T = _corner_setup()
    cam = _cam(64, 48, 40.0)
    d, c = O.scan_image(S.range_image(scene, cam, T, 0, noise_rel=0.0))
    out = O.align_cost(mesh, cam, T, d, c, eps=1.0)
    ev = np.linalg.eigvalsh(out["jtj"])
    assert ev[0] > 1e-6 * ev[-1], "box corner constrains all six directions"
    plane = S.plane_mesh(16, 8.0)
    camp = _cam(64, 48, 40.0)
    dp = O.render(plane, camp, _identity())["z"].reshape(48, 64).astype(np.float32)
    d2, c2 = O.scan_image(dp)
    outp = O.align_cost(plane, camp, _identity(), d2, c2, eps=1.0)
    evp = np.linalg.eigvalsh(outp["jtj"])
    assert np.sum(evp > 1e-9 * evp[-1]) == 3, evp


def test_gauss_newton_converges_on_box_corner(oracle_mod):
    """Noiseless box corner, start 2 cm / 1 deg off, eps large: Gauss-Newton on
    E_soft's residuals reaches the true pose to 1e-9 within 10 iterations."""
    O = oracle_mod
    scene, mesh, T_true = _corner_setup()
    cam = _cam(64, 48, 40.0)
    _, c = O.scan_image(S.range_image(scene, cam, T_true, 0, noise_rel=0.0))
    d = S.analytic_depth(scene, cam, T_true)      # FP64 scan depths: no float32 rounding floor
    rng = np.random.default_rng(2)
    T = S.perturb(T_true, rng, 0.02, np.deg2rad(1.0), fixed=True)
    for it in range(10):
        out = O.align_cost(mesh, cam, T, d, c, eps=1.0)
        T = O.retract(T, O.gn_step(out))
        err = max(np.abs(T[:, 3] - T_true[:, 3]).max(), np.abs(T[:, :3] - T_true[:, :3]).max())
        if err < 1e-9:
            break
    assert err < 1e-9, (it, err)


# ---------------------------------------------------------------- SE(3)

def test_se3_exp_against_scipy(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    for _ in range(20):
        w = rng.normal(size=3) * rng.choice([1e-10, 1e-3, 0.5, 2.0])
        v = rng.normal(size=3)
        E = O.se3_exp(np.concatenate([v, w]))
        np.testing.assert_allclose(E[:3, :3], Rotation.from_rotvec(w).as_matrix(), atol=1e-13)
        # exp(delta) exp(-delta) = I
        np.testing.assert_allclose(E @ O.se3_exp(-np.concatenate([v, w])), np.eye(4), atol=1e-12)
    np.testing.assert_allclose(O.se3_exp(np.array([1.0, 2.0, 3.0, 0, 0, 0]))[:3, 3], [1, 2, 3])
    # rotation about z by theta, translation along the rotation axis is unchanged
    th = 0.7
    E = O.se3_exp(np.array([0, 0, 2.0, 0, 0, th]))
    np.testing.assert_allclose(E[:3, :3], [[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]], atol=1e-15)
    np.testing.assert_allclose(E[:3, 3], [0, 0, 2.0], atol=1e-15)


# ---------------------------------------------------------------- meshify

def test_meshify_counts_and_classes(oracle_mod):
    O = oracle_mod
    cam = _cam(64, 48, 52.5)
    for s in (1, 3, 4, 8):
        depth = np.full((48, 64), 1.0, np.float32)
        xyz, tri, cls = O.meshify(depth, cam, _identity(), s, max_edge=0.1 * max(s, 1))
        gw, gh = -(-64 // s), -(-48 // s)
        assert len(tri) == 2 * (gw - 1) * (gh - 1)
        assert (cls == O.FO).all()
    # all no-return: everything free-unknown at z_max
    xyz, tri, cls = O.meshify(np.zeros((48, 64), np.float32), cam, _identity(), 4)
    assert (cls == O.FU).all() and np.allclose(xyz[:, 2], 8.0)
    # dead pixels drop their quads
    depth = np.full((48, 64), 1.0, np.float32); depth[8, 8] = np.nan
    _, tri, _ = O.meshify(depth, cam, _identity(), 4)
    assert len(tri) == 2 * (15 * 11 - 4)      # node (2,2) is dead: its four quads go


def test_meshify_depth_step_marks_spanning_quads(oracle_mod):
    O = oracle_mod
    cam = _cam(64, 48, 525.0)                # 4 px at 1.5 m is 1.1 cm: only the step exceeds 0.1 m
    depth = np.full((48, 64), 1.0, np.float32)
    depth[:, 32:] = 1.5                      # a 0.5 m step between columns 31 and 32
    xyz, tri, cls = O.meshify(depth, cam, _identity(), 4, max_edge=0.1)
    gw = 16
    j = tri[:, 0] % gw                        # quad column of each triangle (n00 = i*gw + j)
    spans = (j * 4 < 32) & ((j + 1) * 4 >= 32)
    assert (cls[spans] == O.FU).all()
    assert (cls[~spans] == O.FO).all()


def test_meshify_vertices_reproject_to_pixel_centres(oracle_mod):
    O = oracle_mod
    w = configs.tiny()
    cam = w.cam
    xyz, tri, cls = O.meshify(w.scan_depth, cam, w.T_true, 2)
    R, t = w.T_true[:, :3], w.T_true[:, 3]
    used = np.unique(tri)
    Xc = (xyz[used].astype(np.float64) - t) @ R
    u = cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx
    v = cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy
    gw = -(-cam.width // 2)
    np.testing.assert_allclose(u, (used % gw) * 2, atol=1e-4)
    np.testing.assert_allclose(v, (used // gw) * 2, atol=1e-4)


def test_meshify_smoothing_keeps_edges_and_reduces_noise(oracle_mod):
    """Node smoothing (radius R): on a noisy frontal plane the node depths'
    spread drops by about the window side 2R+1 (mean of (2R+1)^2 independent
    samples); across a 2 m / 3 m depth step no pixel of the other side enters
    a node's mean, so noise-free step nodes keep their depth exactly."""
    O = oracle_mod
    cam = _cam(96, 64, 60.0)
    rng = np.random.default_rng(11)
    sigma, R = 0.01, 3
    noisy = (2.0 + sigma * rng.standard_normal((64, 96))).astype(np.float32)
    raw = O.meshify(noisy, cam, _identity(), 1, max_edge=1.0)[0][:, 2]
    smooth = O.meshify(noisy, cam, _identity(), 1, max_edge=1.0, smooth_radius=R)[0][:, 2]
    inner = np.zeros((64, 96), bool); inner[R:-R, R:-R] = True
    ratio = raw[inner.ravel()].std() / smooth[inner.ravel()].std()
    assert 0.85 * (2 * R + 1) < ratio < 1.15 * (2 * R + 1), ratio
    step = np.full((64, 96), 2.0, np.float32); step[:, 48:] = 3.0
    z = O.meshify(step, cam, _identity(), 4, max_edge=1.0, smooth_radius=R)[0][:, 2]
    np.testing.assert_array_equal(np.sort(np.unique(z)), np.array([2.0, 3.0], np.float32))


def test_scan_image_classes(oracle_mod):
    O = oracle_mod
    z = np.array([[1.0, 0.0, np.nan, np.inf, 9.0, 0.2, -1.0, 8.0]], np.float32)
    d, c = O.scan_image(z, z_min=0.5, z_max=8.0)
    assert list(c[0]) == [O.FO, O.FU, O.NONE, O.FU, O.FU, O.NONE, O.NONE, O.FO]
    assert d[0, 1] == 8.0 and d[0, 4] == 8.0 and np.isnan(d[0, 2])


# ---------------------------------------------------------------- contract, brute force in exact arithmetic

def _f32(x):
    return np.float32(x)


def _round_f32(q: Fraction) -> np.float32:
    """Correctly rounded (ties to even) float32 of an exact rational."""
    d = float(q)                       # correctly rounded to double
    f = np.float32(d)
    if Fraction(float(f)) == q:
        return f
    # neighbours of f and the one nearest to q (ties to even mantissa)
    lo = np.nextafter(f, np.float32(-np.inf)); hi = np.nextafter(f, np.float32(np.inf))
    cands = [lo, f, hi]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - q), int(np.array(c).view(np.uint32)) & 1))
    return np.float32(best)


def _fmaf(a, b, c):
    return _round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_contract_snap_exact_arithmetic(oracle_mod):
    """Re-derive the snapped screen vertices of the tiny room's triangles with
    exact rational arithmetic rounded to float32 at each step of the contract,
    and compare with the C oracle's sub-triangles (unclipped ones)."""
    O = oracle_mod
    w = configs.tiny()
    xyz, tri, cls = w.map_mesh
    T = w.poses[0]
    cam = w.cam
    subs = O.contract_subtriangles(w.map_mesh, cam, T)
    R32 = np.array([[_f32(T[j, i]) for j in range(3)] for i in range(3)], dtype=np.float32)
    rng = np.random.default_rng(0)
    checked = 0
    for row in subs[rng.choice(len(subs), min(60, len(subs)), replace=False)]:
        t = int(row[0])
        pts = []
        for k in range(3):
            Xw = xyz[tri[t, k]]
            d = [_round_f32(Fraction(float(Xw[j])) - Fraction(float(T[j, 3]))) for j in range(3)]
            Xc = [_fmaf(R32[i, 2], d[2], _fmaf(R32[i, 1], d[1], _round_f32(Fraction(float(R32[i, 0])) * Fraction(float(d[0]))))) for i in range(3)]
            if Xc[2] < _f32(cam.z_near):
                break
            inv = _round_f32(Fraction(1) / Fraction(float(Xc[2])))
            u = _fmaf(_round_f32(Fraction(float(_f32(cam.fx))) * Fraction(float(Xc[0]))), inv, _f32(cam.cx))
            v = _fmaf(_round_f32(Fraction(float(_f32(cam.fy))) * Fraction(float(Xc[1]))), inv, _f32(cam.cy))
            pts.append((int(np.rint(np.float32(u) * np.float32(256))), int(np.rint(np.float32(v) * np.float32(256)))))
        else:
            got = {(int(row[1 + 2 * j]), int(row[2 + 2 * j])) for j in range(3)}
            assert got == set(pts)
            checked += 1
    assert checked > 20


def test_table_weights_as_printed_give_e_table(oracle_mod):
    """Table I's printed values as cell weights reproduce E(X) exactly, and a
    weight vector is linear in the cell counts."""
    O = oracle_mod
    w = configs.tiny()
    mesh = w.map_mesh
    d, c = O.scan_image(w.scan_depth, w.z_min, w.z_max)
    out = O.align_cost(mesh, w.cam, w.poses[0], d, c, eps=0.1)
    t = out["terms"]
    assert O.table_cost_weighted(t, O.TABLE_WEIGHTS) == out["e_table"]
    rng = np.random.default_rng(8)
    wt = rng.normal(size=9)
    np.testing.assert_allclose(O.table_cost_weighted(t, wt), out["counts"] @ wt, rtol=1e-12)
    assert (np.sign(O.TABLE_WEIGHTS[:6]) == np.array([-1, 1, -1, 1, -1, 1])).all()
