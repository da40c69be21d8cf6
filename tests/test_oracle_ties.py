"""Pins of the oracle's depth tie-break, runner-up depth and the per-pixel
flags that decide which pixels are exempt from parity (CPU only).

Each expected value is a closed form: the depth of a fronto-parallel plane
z = c seen from the identity pose is c at every pixel, the depth of the
floor plane y = h is h / r_y, and the flag thresholds are the ones the
parity rules state (depth near-tie: runner-up within 1e-6 relative; far-plane
tie: within 1e-6 relative of z_far; grazing: |n^ . r^| < 1e-2; Table I
threshold tie: the decision lies within 1e-5 relative of a threshold).  A
plausible mistake in the oracle's tie-break (highest id winning, the
runner-up never replaced, a flag with the wrong side of its threshold)
fails one of these tests.
"""
import numpy as np
import pytest

from workloads import scenes as S


def _identity():
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    return T


def _cam(W=24, H=18, f=20.0, zn=0.1, zf=16.0):
    return S.Camera(f, f, (W - 1) / 2, (H - 1) / 2, W, H, zn, zf)


def _quad(z, half=8.0):
    """Two triangles of the fronto-parallel square |x|, |y| <= half * z / 8 at depth z."""
    s = np.float32(half * z / 8.0)
    z32 = np.float32(z)
    xyz = np.array([[-s, -s, z32], [s, -s, z32], [s, s, z32], [-s, s, z32]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return xyz, tri


def _mesh(parts):
    """Union of (xyz, tri) parts in the given order; ids follow that order."""
    xyz, tri, off = [], [], 0
    for v, t in parts:
        xyz.append(v); tri.append(t + off); off += len(v)
    t = np.concatenate(tri).astype(np.int32)
    return np.concatenate(xyz), t, np.zeros(len(t), np.uint8)


@pytest.mark.parametrize("mode", ["contract", "exact"])
def test_duplicate_triangles_lowest_id_wins(oracle_mod, mode):
    """The same square twice: every covered pixel is won by the lower id of
    the two copies, its runner-up depth equals its depth exactly, and it is
    flagged as a near-tie.  The copies are placed so that the higher id
    comes first in one test and the lower in the other (ids are positions)."""
    O = oracle_mod
    cam = _cam()
    v, t = _quad(2.0)
    other_v, other_t = _quad(5.0)                      # a farther square behind, never the winner
    for order in ((v, t), (other_v, other_t), (v, t)), ((other_v, other_t), (v, t), (v, t)):
        mesh = _mesh(order)
        ids_of_near = [k for k, (pv, _) in enumerate(order) if pv is v]
        out = O.render(mesh, cam, _identity(), mode=mode)
        hit = out["id"] >= 0
        assert hit.sum() > 0.5 * cam.width * cam.height
        # the near square's triangles of the first copy have ids 2*k, 2*k+1
        first = 2 * min(ids_of_near)
        assert set(np.unique(out["id"][hit])) <= {first, first + 1}, np.unique(out["id"][hit])
        np.testing.assert_array_equal(out["z"][hit], np.float64(np.float32(2.0)))
        np.testing.assert_array_equal(out["z2"][hit], out["z"][hit])
        assert O.flags(out, cam)["near_tie"][hit].all()


@pytest.mark.parametrize("mode", ["contract", "exact"])
def test_runner_up_is_the_next_plane(oracle_mod, mode):
    """Two parallel squares at z_a < z_b: the nearer wins and the runner-up
    depth is exactly z_b, whichever of the two has the lower id."""
    O = oracle_mod
    cam = _cam()
    za, zb = 2.0, 3.0
    for parts in ([_quad(za), _quad(zb)], [_quad(zb), _quad(za)]):
        mesh = _mesh(parts)
        near_first = parts[0][0][0, 2] == np.float32(za)
        out = O.render(mesh, cam, _identity(), mode=mode)
        hit = out["id"] >= 0
        assert hit.any()
        np.testing.assert_array_equal(out["z"][hit], za)
        # one covering triangle per square; the exact mode's inclusive edge
        # test also lets both triangles of a square cover its diagonal, where
        # the sibling at the same depth is the runner-up
        two = out["ncov"] == 2
        if mode == "contract":
            assert (two == hit).all()
        assert two.sum() > 0.9 * hit.sum()
        np.testing.assert_array_equal(out["z2"][hit & two], zb)
        np.testing.assert_array_equal(out["z2"][hit & ~two], za)
        assert ((out["id"][hit] < 2) == near_first).all()
        assert not O.flags(out, cam)["near_tie"][hit & two].any()


@pytest.mark.parametrize("rel,tie", [(0.0, True), (2.5e-7, True), (7.5e-7, True), (1.3e-6, False), (4e-6, False)])
def test_near_tie_threshold(oracle_mod, rel, tie):
    """Runner-up z_b = z_a (1 + rel) (both exact float32 depths): the pixel is
    a depth near-tie iff z_b - z_a <= 1e-6 z_a."""
    O = oracle_mod
    cam = _cam()
    za = 2.0
    zb = float(np.float32(za * (1.0 + rel)))
    expect = (zb - za) <= 1e-6 * za
    assert expect == tie                               # the chosen depths sit on the intended side
    mesh = _mesh([_quad(za), _quad(zb)])
    out = O.render(mesh, cam, _identity())
    hit = out["id"] >= 0
    np.testing.assert_array_equal(out["z2"][hit], zb)
    assert (O.flags(out, cam)["near_tie"][hit] == tie).all()


@pytest.mark.parametrize("rel,hit_expected,tie", [(0.0, True, True), (-5e-7, True, True), (-4e-6, True, False),
                                                  (5e-7, False, True), (4e-6, False, False)])
def test_far_plane_tie(oracle_mod, rel, hit_expected, tie):
    """A wall at z_far (1 + rel), exact coverage: beyond z_far it is not
    drawn but its depth is the runner-up; within 1e-6 relative of z_far
    either way it is a far-plane tie."""
    O = oracle_mod
    cam = _cam()
    zf = float(np.float32(cam.z_far))
    zw = float(np.float32(zf * (1.0 + rel)))
    mesh = _mesh([_quad(zw)])
    out = O.render(mesh, cam, _identity(), mode="exact")
    covered = out["ncov"] > 0
    assert covered.sum() > 0.5 * cam.width * cam.height
    assert ((out["id"] >= 0)[covered] == hit_expected).all()
    if hit_expected:
        np.testing.assert_array_equal(out["z"][covered], zw)
    else:
        assert np.isnan(out["z"][covered]).all()
        np.testing.assert_array_equal(out["z2"][covered], zw)
    assert (O.flags(out, cam)["far_tie"][covered] == tie).all()


def test_far_plane_tie_tilted_wall_contract(oracle_mod):
    """Contract coverage of a wall z = z_far + a x that crosses the far plane:
    pixels whose closed-form depth 16 / (1 - a r_x) is beyond z_far are
    covered but empty, and exactly those within 1e-6 relative of z_far on
    either side are far-plane ties."""
    O = oracle_mod
    cam = _cam(W=64, H=8, f=40.0)
    a = 2e-6                                            # about 1e-6 relative per pixel
    zf = float(np.float32(cam.z_far))
    xs = np.array([-20.0, 20.0], np.float32)
    xyz = np.array([[xs[0], -10, zf + a * xs[0]], [xs[1], -10, zf + a * xs[1]], [xs[1], 10, zf + a * xs[1]],
                    [xs[0], 10, zf + a * xs[0]]], np.float32)
    mesh = (xyz, np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.zeros(2, np.uint8))
    out = O.render(mesh, cam, _identity())
    r = O.rays(cam, out["pixels"])
    # plane through the float32 vertices: z = c0 + a32 x, with the x-slope of the rounded vertices
    a32 = (float(xyz[1, 2]) - float(xyz[0, 2])) / (float(xyz[1, 0]) - float(xyz[0, 0]))
    c0 = float(xyz[0, 2]) - a32 * float(xyz[0, 0])
    z_cf = c0 / (1.0 - a32 * r[:, 0])
    cov = out["ncov"] > 0
    assert cov.all()
    hit = out["id"] >= 0
    np.testing.assert_array_equal(hit, z_cf <= zf)
    np.testing.assert_allclose(np.where(hit, out["z"], out["z2"]), z_cf, rtol=1e-12)
    expect = np.abs(z_cf - zf) <= 1e-6 * zf
    clear = np.abs(np.abs(z_cf - zf) - 1e-6 * zf) > 1e-9
    far = O.flags(out, cam)["far_tie"]
    assert ((far == expect) | ~clear).all()
    assert expect.any() and (~expect & hit).any() and (~expect & ~hit).any()


def test_grazing_flag_closed_form(oracle_mod):
    """The floor y = h seen from the identity pose: a pixel's |n^ . r^| is
    |r_y| / |r|, and it is flagged grazing iff that is below 1e-2."""
    O = oracle_mod
    # horizon half a pixel above row 0; with f = 400 px and the floor 0.1 m
    # below the camera, row 4 (|n^ . r^| ~ 0.0087, 11 m away) is grazing
    cam = S.Camera(400.0, 400.0, 31.5, 0.5, 64, 48, 0.1, 16.0)
    h = 0.1
    k = np.array([-30.0, -1.0, 1.0, 30.0], np.float32)
    xyz = np.array([[k[0], h, 0.2], [k[3], h, 0.2], [k[3], h, 15.9], [k[0], h, 15.9]], np.float32)
    mesh = (xyz, np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.zeros(2, np.uint8))
    out = O.render(mesh, cam, _identity(), mode="exact")
    hit = out["id"] >= 0
    r = O.rays(cam, out["pixels"])
    cosang = np.abs(r[:, 1]) / np.linalg.norm(r, axis=1)
    np.testing.assert_allclose(out["z"][hit], float(np.float32(h)) / r[hit, 1], rtol=1e-12)
    graz = O.flags(out, cam)["grazing"]
    clear = np.abs(cosang - 1e-2) > 1e-9
    expect = hit & (cosang < 1e-2)
    assert ((graz == expect) | ~clear).all()
    assert expect.sum() > 0 and (hit & ~expect).sum() > 0   # both sides are present


# ---------------------------------------------------------------- Table I threshold ties

def _terms_at(O, cam, c_r, c_s, d_r, d_s, eps):
    """pixel_terms of a synthetic render: every pixel at the principal point
    column/row grid of a fronto-parallel plane (|n^ . r| = 1 at the centre
    pixel, so e = dz there)."""
    n = len(d_r)
    pix = np.full(n, (cam.height // 2) * cam.width + cam.width // 2, np.int64)
    rend = dict(pixels=pix, id=np.where(np.asarray(c_r) == O.NONE, -1, 0).astype(np.int32),
                z=np.asarray(d_r, np.float64), nrm=np.tile([0.0, 0.0, -1.0], (n, 1)))
    mesh_cls = np.array([c_r[0] if c_r[0] != O.NONE else O.FO], np.uint8)
    sd = np.full(cam.width * cam.height, np.nan)
    sc = np.full(cam.width * cam.height, O.NONE, np.uint8)
    terms = []
    for k in range(n):
        sd[pix[k]] = d_s[k]
        sc[pix[k]] = c_s[k]
        one = {kk: (vv[k:k + 1] if isinstance(vv, np.ndarray) else vv) for kk, vv in rend.items()}
        terms.append(O.pixel_terms(one, mesh_cls, sd, sc, cam, eps))
    return {k: np.concatenate([t[k] for t in terms]) for k in terms[0]}


def test_threshold_ties_closed_form(oracle_mod):
    """Depth differences placed at 1e-7 and 1e-3 relative of each Table I
    threshold: FO/FO at |dz| = eps, FO/FU and FU/FO at dz = 0, and the edge
    of the E_soft band |r| = eps on the one-sided cells, at a depth of 2 m
    (tolerance 2e-5 m).  Only the 1e-7 ones are threshold ties; ignored cells
    never are."""
    O = oracle_mod
    cam = S.Camera(20.0, 20.0, 12.0, 9.0, 25, 19, 0.1, 16.0)   # integer principal point: ray (0, 0, 1)
    eps = 0.1
    ds = 2.0
    cases = []
    for k in (1e-7, -1e-7, 1e-3, -1e-3):
        for sgn in (1.0, -1.0):
            cases.append((O.FO, O.FO, ds + sgn * eps * (1 + k), ds, abs(k) < 1e-6))
        cases.append((O.FO, O.FU, ds + k * ds, ds, abs(k) < 1e-6))
        cases.append((O.FU, O.FO, ds + k * ds, ds, abs(k) < 1e-6))
        cases.append((O.FO, O.FU, ds - eps * (1 + k), ds, abs(k) < 1e-6))      # band edge, r = dz < 0
        cases.append((O.FU, O.FO, ds + eps * (1 + k), ds, abs(k) < 1e-6))      # band edge, r = dz > 0
        cases.append((O.FU, O.FU, ds + eps * (1 + k), ds, False))             # ignored cell
        cases.append((O.NONE, O.FO, ds, ds, False))                           # ignored cell
    for c_r, c_s, d_r, d_s, tie in cases:
        t = _terms_at(O, cam, [c_r], [c_s], [d_r], [d_s], eps)
        assert bool(O.threshold_ties(t, eps)[0]) == tie, (c_r, c_s, d_r - d_s, tie)


def test_threshold_ties_are_sufficient(oracle_mod):
    """Outside the flagged pixels, moving dz by the depth tolerance never
    changes the Table I cell or whether |r| < eps: the flag covers every
    decision the float32 depth could flip."""
    O = oracle_mod
    cam = S.Camera(20.0, 20.0, 12.0, 9.0, 25, 19, 0.1, 16.0)
    eps = 0.1
    rng = np.random.default_rng(0)
    n = 400
    c_r = rng.choice([O.FO, O.FU], n)
    c_s = rng.choice([O.FO, O.FU], n)
    base = rng.choice([0.0, eps, -eps], n)
    d_s = rng.uniform(0.5, 8.0, n)
    d_r = d_s + base + rng.normal(0, 1e-5, n) * d_s
    t = _terms_at(O, cam, c_r, c_s, d_r, d_s, eps)
    flagged = O.threshold_ties(t, eps)
    assert flagged.any() and (~flagged).any()
    scale = O.DEPTH_REL * np.maximum(np.abs(d_r), np.abs(d_s))
    for sgn in (-1.0, 1.0):
        t2 = _terms_at(O, cam, c_r, c_s, d_r + sgn * 0.999 * scale, d_s, eps)
        same = (t2["cell"] == t["cell"]) & ((np.abs(t2["r"]) < eps) == (np.abs(t["r"]) < eps))
        assert same[~flagged].all()


def test_icp_tol_ties_closed_form(oracle_mod):
    """The association decision |Z_M - Z_1| < tol is a tie iff it lies within
    1e-5 relative of tol, and only pixels that see a model surface count."""
    O = oracle_mod
    tol = 0.1
    z1 = np.full(8, 2.0)
    k = np.array([1e-7, -1e-7, 1e-3, -1e-3, 1e-7, -1e-7, 1e-3, 0.0])
    sgn = np.array([1, 1, 1, 1, -1, -1, -1, 1], np.float64)
    zM = z1 + sgn * tol * (1 + k)
    model = np.array([True] * 7 + [False])
    terms = dict(model=model, zM=zM, z1=z1, dz=zM - z1)
    got = O.icp_tol_ties(terms, tol)
    np.testing.assert_array_equal(got, model & (np.abs(k) < 1e-6))
