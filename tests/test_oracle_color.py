"""Pins of the oracle's color term against closed forms: a fronto-parallel
plane of two colors seen from the identity pose, where every pixel's
triangle side, Table I cell and color decision follow from the geometry.
They fix which pixels correspond (only the FO/FO reward cell), which
triangle's color a pixel takes, that the threshold is inclusive and taken in
float32, and which pixels are left out (scan or map color NaN, penalized or
unscored depth cells).  CPU only."""
import numpy as np

from workloads import scenes as S

W, H = 64, 48
LEFT = 32                       # columns u <= 31 see x < 0 (cx = 31.5: no ray meets x = 0)


def _setup(oracle_mod):
    O = oracle_mod
    xyz, tri, cls = S.plane_mesh(n_per_side=8, extent=4.0, z0=2.0, slope=(0.0, 0.0))
    cam = S.Camera(40.0, 40.0, 31.5, 23.5, W, H, 0.1, 16.0)
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    left = xyz[tri].mean(axis=1)[:, 0] < 0
    assert left.sum() == len(tri) // 2
    tri_color = np.where(left, np.float32(0.25), np.float32(0.75)).astype(np.float32)
    rend = O.render((xyz, tri), cam, T)
    assert (rend["id"] >= 0).all() and (rend["z"] == 2.0).all()
    side_left = left[rend["id"]].reshape(H, W)
    u = np.arange(W)
    assert (side_left == (u < LEFT)[None, :]).all()
    return O, (xyz, tri, cls), cam, T, rend, tri_color


def _cells(O, rend, cls, depth, tri_color, scan_color, tol, eps=0.1):
    d_s, c_s = O.scan_image(depth)
    terms = O.pixel_terms(rend, cls, d_s, c_s, S.Camera(40.0, 40.0, 31.5, 23.5, W, H, 0.1, 16.0), eps)
    return terms, O.color_cells(terms, rend, tri_color, scan_color, tol)


def test_color_threshold_inclusive_and_side(oracle_mod):
    O, mesh, cam, T, rend, tri_color = _setup(oracle_mod)
    depth = np.full((H, W), 2.0, np.float32)
    # |0.25 - 0.5| = |0.75 - 0.5| = 0.25: both sides exactly at the threshold
    terms, cells = _cells(O, rend, mesh[2], depth, tri_color, np.full((H, W), 0.5, np.float32), 0.25)
    assert (terms["cell"] == 0).all()
    assert O.color_counts(cells) == (W * H, 0)
    # one float32 step above 0.5 (2^-10 here): the left side falls just outside
    s = np.float32(0.5 + 2.0 ** -10)
    _, cells = _cells(O, rend, mesh[2], depth, tri_color, np.full((H, W), s, np.float32), 0.25)
    assert O.color_counts(cells) == ((W - LEFT) * H, LEFT * H)
    assert (cells.reshape(H, W)[:, :LEFT] == O.COLOR_PENALTY).all()
    # scan colors 0.25 on columns u < 20, 0.75 elsewhere, tol 0.1
    sc = np.where(np.arange(W)[None, :] < 20, np.float32(0.25), np.float32(0.75)) * np.ones((H, 1), np.float32)
    _, cells = _cells(O, rend, mesh[2], depth, tri_color, sc.astype(np.float32), 0.1)
    assert O.color_counts(cells) == ((20 + W - LEFT) * H, (LEFT - 20) * H)


def test_color_only_on_corresponding_pixels(oracle_mod):
    O, mesh, cam, T, rend, tri_color = _setup(oracle_mod)
    depth = np.full((H, W), 2.0, np.float32)
    depth[0:5] = 2.5            # FO/FO penalty (|dz| = 0.5 > eps): not corresponding
    depth[5:8] = 0.0            # no return: FO/FU
    depth[10] = np.nan          # dead scan pixel: ignored by Table I
    sc = np.full((H, W), 0.5, np.float32)
    sc[8:10] = np.nan           # no scan color
    tc = tri_color.copy()
    terms, cells = _cells(O, rend, mesh[2], depth, tc, sc, 0.25)
    assert O.color_counts(cells) == (W * (H - 11), 0)
    assert (cells.reshape(H, W)[:11] == O.COLOR_NONE).all()
    # map color NaN on the left triangles: their pixels drop out
    tc[tc == np.float32(0.25)] = np.nan
    _, cells = _cells(O, rend, mesh[2], depth, tc, sc, 0.25)
    assert O.color_counts(cells) == ((W - LEFT) * (H - 11), 0)
    # the same scan with the depth 2.05 (inside eps): every cell still FO/FO reward
    terms, cells = _cells(O, rend, mesh[2], np.full((H, W), 2.05, np.float32), tri_color, sc, 0.25)
    assert (terms["cell"] == 0).all()
    assert O.color_counts(cells) == (W * (H - 2), 0)


def test_color_weighted_cost(oracle_mod):
    """Weights (Table I's values, -1 per rewarded, +1 per penalized color)
    give E(X) plus penalties minus rewards; zero color weights give E(X)."""
    O, mesh, cam, T, rend, tri_color = _setup(oracle_mod)
    depth = np.full((H, W), 2.0, np.float32)
    depth[0:6] = 2.5
    sc = np.full((H, W), np.float32(0.5 + 2.0 ** -10), np.float32)
    terms, cells = _cells(O, rend, mesh[2], depth, tri_color, sc, 0.25)
    e_table = int(terms["s"].sum())
    assert e_table == W * 6 - W * (H - 6)
    w = np.concatenate([O.TABLE_WEIGHTS, [-1.0, 1.0]])
    nr, npen = O.color_counts(cells)
    assert (nr, npen) == ((W - LEFT) * (H - 6), LEFT * (H - 6))
    assert O.table_color_cost_weighted(terms, cells, w) == e_table - nr + npen
    assert O.table_color_cost_weighted(terms, cells, np.concatenate([O.TABLE_WEIGHTS, [0.0, 0.0]])) == e_table


def test_color_generators():
    """The synthetic intensity: inside [0.05, 0.95]; per-triangle albedo at
    the centroid; the intensity image NaN exactly where the range image has
    no return within range (no noise, no dropouts)."""
    a = S.albedo(np.random.default_rng(0).uniform(-10, 10, (1000, 3)))
    assert a.min() >= 0.05 - 1e-12 and a.max() <= 0.95 + 1e-12
    xyz = np.array([[0, 0, 0], [0.35, 0, 0], [0, 0.45, 0]], np.float32)
    assert np.isclose(S.triangle_albedo(xyz, np.array([[0, 1, 2]]))[0], S.albedo(xyz.mean(0)), atol=1e-7)
    scene = S.random_box_room(2, (4.0, 4.0, 2.5), 4, )
    cam = S.Camera(30.0, 30.0, 15.5, 11.5, 32, 24, 0.1, 16.0)
    c = 0.5 * (scene.room_lo + scene.room_hi)
    T = S.look_pose(np.array([c[0], c[1], 1.2]), 0.3, 0.0)
    I = S.intensity_image(scene, cam, T, 1, noise=0.0)
    z = S.range_image(scene, cam, T, 1, noise_rel=0.0)
    assert (np.isnan(I) == (z == 0)).all()


def test_color_of_the_triangle_each_pixel_sees(oracle_mod):
    """Every triangle its own color (id / 256, exact in float32) and each scan
    pixel the color of the triangle found from the geometry alone: the pixel
    meets the plane z = 2 at (x, y) = 2 r, inside the unit quad (i, j) =
    floor((x, y) + 4), whose first triangle (id 8 i + j) holds the part above
    its diagonal and whose second (id 64 + 8 i + j) the rest (cy = 23.25 keeps
    every ray off the diagonals).  With tol = 0 every corresponding pixel is
    rewarded only if the oracle takes the color of exactly that triangle."""
    O = oracle_mod
    xyz, tri, cls = S.plane_mesh(n_per_side=8, extent=4.0, z0=2.0, slope=(0.0, 0.0))
    cam = S.Camera(40.0, 40.0, 31.5, 23.25, W, H, 0.1, 16.0)
    T = np.zeros((3, 4)); T[:, :3] = np.eye(3)
    tri_color = (np.arange(len(tri)) / 256.0).astype(np.float32)
    u, v = np.meshgrid(np.arange(W), np.arange(H))
    x, y = (u - 31.5) / 20.0, (v - 23.25) / 20.0
    i, j = np.floor(x + 4).astype(int), np.floor(y + 4).astype(int)
    upper = (y + 4 - j) > (x + 4 - i)
    want = np.where(upper, 8 * i + j, 64 + 8 * i + j)
    assert len(np.unique(want)) > 8
    rend = O.render((xyz, tri), cam, T)
    d_s, c_s = O.scan_image(np.full((H, W), 2.0, np.float32))
    terms = O.pixel_terms(rend, cls, d_s, c_s, cam, 0.1)
    cells = O.color_cells(terms, rend, tri_color, tri_color[want], 0.0)
    assert O.color_counts(cells) == (W * H, 0)
    shifted = O.color_cells(terms, rend, tri_color, tri_color[(want + 1) % len(tri)], 0.0)
    assert O.color_counts(shifted) == (0, W * H)
