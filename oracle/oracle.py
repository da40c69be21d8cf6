"""FP64 oracle of the RenderMap pose-scoring path (arXiv 1702.06813).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product library never
imports, links or calls anything here, and this module shares no code with it.

Pieces, each following the paper:
  * scan image and meshification (Sec. IV-A) and the brute-force z-buffer
    R(T(X)) of Eq. (1): the C file ``rm_oracle.c`` next to this module;
  * the per-pixel comparison C of Table I (Sec. IV-B) with epsilon = 0.1 m,
    and the total error E(X) = sum over pixels (Sec. IV-B);
  * E_soft, a continuous surrogate of E(X) (the paper invites reshaping the
    per-pixel cost, Sec. IV-C) with its se(3) gradient and the Gauss-Newton
    blocks J^T J / J^T r; and SE(3) exp for pose increments;
  * the render-accelerated point-to-plane ICP of Sec. V: downsampling,
    Gaussian smoothing and the depth-image normals of Eq. (2), per-vertex
    normals, projective association with a depth tolerance, the cost
    C = sum |Z_M - Z_1| and the point-to-plane Gauss-Newton blocks (readings
    in the section below).

E_soft (a project definition; the paper optimizes E derivative-free):
    rho_p = 2 * min(r_p^2 / eps^2, 1) - 1   on the three scored cells,
    rho_p = 0                              on ignored cells, with
    r_p = e_p          (map FO, scan FO)
    r_p = min(e_p, 0)  (map FO, scan FU: penalty side is dz <= 0)
    r_p = max(e_p, 0)  (map FU, scan FO: penalty side is dz > 0)
    e_p = dz * |n^ . ray|,  dz = d(p_r) - d(p_s)  (Table I),
where n^ is the winning triangle's camera-frame unit normal and
ray = ((u-cx)/fx, (v-cy)/fy, 1): e_p is the signed distance of the scan point
P_s = d(p_s) ray from the plane of the triangle the pixel sees, positive when
the scan point lies on the camera side (the sign of dz).  Measured across the
plane rather than along the ray, it stays bounded where the ray grazes the
triangle; Table I itself still decides on dz.
rho equals -1 where the Table I cell is a reward with r = 0, and +1 once
|r| >= eps.  A pixel is *active* when its residual moves with the pose:
scored, r^2 < eps^2, and (FO/FO, or FO/FU with dz < 0, or FU/FO with dz > 0).
    grad E_soft = (4 / eps^2) * sum_active r_p J_p
    H = sum_active J_p^T J_p ,  b = sum_active r_p J_p
J_p is the derivative of e_p with respect to a right perturbation
T_wc * exp(delta), delta = (upsilon, omega), the winning triangle held fixed:
e_p = m_w . (T_wc P_s) - c_w for the world plane m_w . X = c_w, so
    J_p = [ m ; P_s x m ],   m = n^ oriented towards the camera (m . ray < 0;
                             m = -n^ when n^ . ray = 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "rm_oracle.c"
LIB = HERE / "liboracle.so"

FO, FU, UO, NONE = 0, 1, 2, 3

# Table I cell indices of the per-pose counts
CELL_NAMES = ["FO/FO reward", "FO/FO penalty", "FO/FU reward", "FO/FU penalty",
              "FU/FO reward", "FU/FO penalty", "ignore: scan NaN", "ignore: map NaN or UO",
              "ignore: FU/FU"]

# tolerances that define the flagged pixels (see the tests that use them)
NEAR_TIE_REL = 1e-6       # depth near-tie between the two nearest surfaces
DEPTH_REL = 1e-5          # depth agreement; also the width of a threshold tie
GRAZING_COS = 1e-2        # |n^ . r^| below this: grazing view of the winner


def build(force: bool = False) -> Path:
    """Compile the C part of the oracle with gcc (OpenMP, no FP contraction)."""
    if force or not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
               "-shared", "-fPIC", "-o", str(LIB), str(SRC), "-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class _Cam(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_float), ("z_far", ctypes.c_float)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB.exists():
            build()
        L = ctypes.CDLL(str(LIB))
        P = ctypes.c_void_p
        L.or_num_threads.restype = ctypes.c_int
        L.or_scan_image.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, P, P]
        L.or_meshify.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Cam), P,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 P, P, P, ctypes.c_int64, P]
        L.or_meshify.restype = ctypes.c_int64
        L.or_render.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, ctypes.POINTER(_Cam),
                                ctypes.c_int32, P, ctypes.c_int64, P, P, P, P, P]
        L.or_render.restype = ctypes.c_int64
        L.or_contract_subs.argtypes = [P, P, ctypes.c_int64, P, ctypes.POINTER(_Cam), P, ctypes.c_int64]
        L.or_contract_subs.restype = ctypes.c_int64
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _cam(cam) -> _Cam:
    fx, fy, cx, cy, W, H, zn, zf = cam.astuple() if hasattr(cam, "astuple") else cam
    return _Cam(fx, fy, cx, cy, int(W), int(H), zn, zf)


def _pose(T):
    return np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(12))


# --------------------------------------------------------------------------
# Sec. IV-A: scan image and meshification
# --------------------------------------------------------------------------

def scan_image(depth, z_min=0.5, z_max=8.0):
    """(d_s f32 [H,W], c_s u8 [H,W]) from a range image."""
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = depth.shape
    d = np.empty((H, W), np.float32)
    c = np.empty((H, W), np.uint8)
    lib().or_scan_image(_ptr(depth), H, W, z_min, z_max, _ptr(d), _ptr(c))
    return d, c


def meshify(depth, cam, T_wc, stride, z_min=0.5, z_max=8.0, max_edge=0.1, smooth_radius=0):
    """Interface mesh (xyz f32 [V,3], tri i32 [T,3], cls u8 [T]) of a range image."""
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    H, W = depth.shape
    gh, gw = -(-H // stride), -(-W // stride)
    cap_t = 2 * max(gh - 1, 0) * max(gw - 1, 0)
    xyz = np.empty((gh * gw, 3), np.float32)
    tri = np.empty((max(cap_t, 1), 3), np.int32)
    cls = np.empty(max(cap_t, 1), np.uint8)
    nv = ctypes.c_int64(0)
    c = _cam(cam)
    nt = lib().or_meshify(_ptr(depth), H, W, ctypes.byref(c), _ptr(_pose(T_wc)), stride, smooth_radius,
                          z_min, z_max, max_edge, _ptr(xyz), _ptr(tri), _ptr(cls), cap_t,
                          ctypes.byref(nv))
    assert nt >= 0
    return xyz, tri[:nt].copy(), cls[:nt].copy()


# --------------------------------------------------------------------------
# Eq. (1): brute-force z-buffer
# --------------------------------------------------------------------------

def render(mesh, cam, T_wc, pixels=None, mode="contract"):
    """Z-buffer of ``mesh`` seen from ``T_wc`` at linear ``pixels`` (all if None).

    Returns a dict of per-pixel arrays: z (NaN: no surface), id (-1), z2
    (runner-up depth), ncov (covering triangles), nrm (winner camera-frame
    normal) and the scalar ``dropped`` (sub-triangles beyond the snap range).
    """
    xyz, tri = (np.ascontiguousarray(mesh[0], np.float32), np.ascontiguousarray(mesh[1], np.int32))
    W, H = cam.width, cam.height
    if pixels is None:
        n, pix = W * H, None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.size
    z = np.empty(n); z2 = np.empty(n); nrm = np.empty((n, 3))
    ids = np.empty(n, np.int32); ncov = np.empty(n, np.int32)
    c = _cam(cam)
    dropped = lib().or_render(_ptr(xyz), xyz.shape[0], _ptr(tri), tri.shape[0], _ptr(_pose(T_wc)),
                              ctypes.byref(c), 0 if mode == "contract" else 1, _ptr(pix), n,
                              _ptr(z), _ptr(ids), _ptr(z2), _ptr(ncov), _ptr(nrm))
    return dict(z=z, id=ids, z2=z2, ncov=ncov, nrm=nrm, dropped=int(dropped),
                pixels=np.arange(W * H) if pixels is None else pix)


def contract_subtriangles(mesh, cam, T_wc):
    """The snapped sub-triangles of the rasterization contract for one pose:
    int64 [N, 7] rows (parent id, X0, Y0, X1, Y1, X2, Y2) in 1/256 px."""
    xyz, tri = np.ascontiguousarray(mesh[0], np.float32), np.ascontiguousarray(mesh[1], np.int32)
    cap = 2 * tri.shape[0] + 1
    out = np.empty((cap, 7), np.int64)
    c = _cam(cam)
    ns = lib().or_contract_subs(_ptr(xyz), _ptr(tri), tri.shape[0], _ptr(_pose(T_wc)),
                                ctypes.byref(c), _ptr(out), cap)
    return out[:ns].copy()


def rays(cam, pixels):
    """Camera-frame ray r = ((u-cx)/fx, (v-cy)/fy, 1) of each linear pixel, FP64."""
    u = (pixels % cam.width).astype(np.float64)
    v = (pixels // cam.width).astype(np.float64)
    return np.stack([(u - np.float64(np.float32(cam.cx))) / np.float64(np.float32(cam.fx)),
                     (v - np.float64(np.float32(cam.cy))) / np.float64(np.float32(cam.fy)),
                     np.ones_like(u)], -1)


def flags(rend, cam):
    """Per-pixel flags of a render: near_tie, far_tie, grazing."""
    z, z2 = rend["z"], rend["z2"]
    hit = rend["id"] >= 0
    zf = float(np.float32(cam.z_far))
    with np.errstate(invalid="ignore"):
        near = hit & (z2 - z <= NEAR_TIE_REL * z)
        far = (hit & (z >= zf * (1 - NEAR_TIE_REL))) | (~hit & (z2 <= zf * (1 + NEAR_TIE_REL)))
        r = rays(cam, rend["pixels"])
        n = rend["nrm"]
        cosang = np.abs((n * r).sum(-1)) / (np.linalg.norm(n, axis=-1) * np.linalg.norm(r, axis=-1))
        graz = hit & ~(cosang >= GRAZING_COS)
    return dict(near_tie=near, far_tie=far, grazing=graz)


# --------------------------------------------------------------------------
# Table I and E(X) (Sec. IV-B); E_soft, gradient and Gauss-Newton blocks
# --------------------------------------------------------------------------

def table1(c_r, c_s, dz, eps):
    """Per-pixel Table I value s in {-1, 0, +1} and cell index (CELL_NAMES)."""
    c_r = np.asarray(c_r); c_s = np.asarray(c_s); dz = np.asarray(dz, dtype=np.float64)
    s = np.zeros(dz.shape, np.int64)
    cell = np.full(dz.shape, 8, np.int64)
    with np.errstate(invalid="ignore"):
        ff = (c_r == FO) & (c_s == FO)
        fu = (c_r == FO) & (c_s == FU)
        uf = (c_r == FU) & (c_s == FO)
        pen_ff = np.abs(dz) > eps          # |dz| > eps penalize, |dz| <= eps reward
        pen_fu = dz <= 0                   # penalize if dz <= 0, reward if dz > 0
        pen_uf = dz > 0                    # penalize if dz > 0, reward if dz <= 0
    for m, pen, base in ((ff, pen_ff, 0), (fu, pen_fu, 2), (uf, pen_uf, 4)):
        s[m] = np.where(pen[m], 1, -1)
        cell[m] = base + pen[m].astype(np.int64)
    scan_na = (c_s == NONE) | (c_s == UO)
    map_na = ~scan_na & ((c_r == NONE) | (c_r == UO))
    cell[scan_na] = 6
    cell[map_na] = 7
    return s, cell


def residual(c_r, c_s, dz, g=1.0):
    """E_soft residual r_p from dz and the plane factor g = |n^ . ray|, the
    mask of scored cells and the mask of cells whose residual moves."""
    ff = (c_r == FO) & (c_s == FO)
    fu = (c_r == FO) & (c_s == FU)
    uf = (c_r == FU) & (c_s == FO)
    with np.errstate(invalid="ignore"):
        e = dz * g
        r = np.where(ff, e, np.where(fu, np.minimum(e, 0.0), np.where(uf, np.maximum(e, 0.0), 0.0)))
        moving = ff | (fu & (dz < 0)) | (uf & (dz > 0))
    scored = ff | fu | uf
    return np.where(scored, r, 0.0), scored, moving


def pixel_terms(rend, mesh_cls, scan_d, scan_c, cam, eps):
    """Per-pixel Table I value, E_soft term, residual and Jacobian."""
    pix = rend["pixels"]
    hit = rend["id"] >= 0
    c_r = np.where(hit, np.asarray(mesh_cls)[np.maximum(rend["id"], 0)], NONE)
    d_r = rend["z"]
    d_s = np.asarray(scan_d, np.float64).reshape(-1)[pix]
    c_s = np.asarray(scan_c).reshape(-1)[pix]
    with np.errstate(invalid="ignore"):
        dz = d_r - d_s
    s, cell = table1(c_r, c_s, dz, eps)
    ray = rays(cam, pix)
    n = np.where(hit[:, None], rend["nrm"], 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        nn = np.linalg.norm(n, axis=-1)
        nh = n / np.where(nn > 0, nn, 1.0)[:, None]
        ndr = (nh * ray).sum(-1)
    g = np.abs(ndr)
    r, scored, moving = residual(c_r, c_s, dz, g)
    rho = np.where(scored, 2.0 * np.minimum(r * r / (eps * eps), 1.0) - 1.0, 0.0)
    active = scored & moving & (r * r < eps * eps)
    m = np.where((ndr < 0)[:, None], nh, -nh)
    with np.errstate(invalid="ignore"):
        Ps = np.where(np.isfinite(d_s), d_s, 0.0)[:, None] * ray
        J = np.concatenate([m, np.cross(Ps, m)], -1)
    J = np.where(active[:, None], J, 0.0)
    return dict(s=s, cell=cell, rho=rho, r=r, active=active, J=J, dz=dz, c_r=c_r, c_s=c_s,
                d_r=d_r, d_s=d_s, g=g, ray_norm=np.linalg.norm(ray, axis=-1))


def threshold_ties(terms, eps):
    """Pixels whose Table I decision, or whether their E_soft residual is
    inside the band |r| < eps, lies within the depth tolerance of a threshold."""
    with np.errstate(invalid="ignore"):
        scale = DEPTH_REL * np.fmax(np.abs(terms["d_r"]), np.abs(terms["d_s"]))
        dz = terms["dz"]
        ff = (terms["c_r"] == FO) & (terms["c_s"] == FO)
        one = ((terms["c_r"] == FO) & (terms["c_s"] == FU)) | ((terms["c_r"] == FU) & (terms["c_s"] == FO))
        # |r| = |dz| g: a depth error of scale and a relative error of 1e-6 in g
        band = (ff | one) & (np.abs(np.abs(terms["r"]) - eps) <= scale * terms["g"] + 1e-6 * np.abs(dz) * terms["ray_norm"])
        return (ff & (np.abs(np.abs(dz) - eps) <= scale)) | (one & (np.abs(dz) <= scale)) | band


def reduce_terms(terms, mask=None):
    """E_table, E_soft, 9 cell counts, gradient, J^T r, J^T J, n_active."""
    m = np.ones(terms["s"].shape, bool) if mask is None else np.asarray(mask, bool)
    J = terms["J"][m]
    r = terms["r"][m]
    act = terms["active"][m]
    b = (r[act, None] * J[act]).sum(0)
    H = J[act].T @ J[act]
    return dict(e_table=int(terms["s"][m].sum()), e_soft=float(terms["rho"][m].sum()),
                counts=np.bincount(terms["cell"][m], minlength=9), jtr=b, jtj=H,
                n_active=int(act.sum()))


def align_cost(mesh, cam, T_wc, scan_d, scan_c, eps=0.1, pixels=None, mode="contract"):
    """Cost, gradient and Gauss-Newton blocks of one pose (FP64)."""
    rend = render(mesh, cam, T_wc, pixels, mode)
    terms = pixel_terms(rend, mesh[2], scan_d, scan_c, cam, eps)
    out = reduce_terms(terms)
    out["grad"] = (4.0 / (eps * eps)) * out["jtr"]
    out["terms"] = terms
    out["render"] = rend
    return out


# --------------------------------------------------------------------------
# SE(3)
# --------------------------------------------------------------------------

def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(delta):
    """4x4 exp of delta = (upsilon, omega) (Rodrigues rotation, V-matrix translation)."""
    v = np.asarray(delta[:3], np.float64); w = np.asarray(delta[3:], np.float64)
    th = float(np.linalg.norm(w))
    K = _hat(w)
    if th < 1e-8:
        A, B, C = 1.0 - th * th / 6.0, 0.5 - th * th / 24.0, 1.0 / 6.0 - th * th / 120.0
    else:
        A, B, C = np.sin(th) / th, (1.0 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
    R = np.eye(3) + A * K + B * (K @ K)
    V = np.eye(3) + B * K + C * (K @ K)
    out = np.eye(4)
    out[:3, :3] = R
    out[:3, 3] = V @ v
    return out


def retract(T_wc, delta):
    """T_wc * exp(delta) as a 3x4 matrix."""
    T = np.vstack([np.asarray(T_wc, np.float64).reshape(3, 4), [0, 0, 0, 1]])
    return (T @ se3_exp(delta))[:3]


def gn_step(out, lam=0.0):
    """Levenberg-Marquardt increment delta = -(H + lam diag H)^-1 b."""
    H = out["jtj"]
    A = H + lam * np.diag(np.diag(H))
    return -np.linalg.solve(A, out["jtr"])


def adam_step(grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps_adam=1e-12):
    """One Adam update of a pose increment from the se(3) gradient (Kingma
    and Ba's first and second moment estimates with bias correction):
        m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
        delta = -lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps_adam).
    Returns (delta, m, v) as new arrays; the pose then moves by T exp(delta)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return -lr * mhat / (np.sqrt(vhat) + eps_adam), m, v


def fd_jacobian(mesh, cam, T_wc, pixels, scan_d, scan_c, h=1e-4, mode="contract"):
    """Central finite differences of the unclamped E_soft residual e_p =
    dz |n^ . ray| with respect to the six components of delta.  Returns
    (fd [N,6], stable [N] mask of hit pixels whose winning triangle is the same
    at -h, 0 and +h on every axis, terms at T_wc with every scored pixel inside
    the band)."""
    def terms(T):
        rend = render(mesh, cam, T, pixels, mode)
        t = pixel_terms(rend, mesh[2], scan_d, scan_c, cam, 1e30)
        return rend, t, t["dz"] * t["g"]
    base, t0, _ = terms(T_wc)
    fd = np.zeros((len(pixels), 6))
    stable = base["id"] >= 0
    for k in range(6):
        e = np.zeros(6); e[k] = h
        rp, _, ep = terms(retract(T_wc, e))
        rm, _, em = terms(retract(T_wc, -e))
        fd[:, k] = (ep - em) / (2 * h)
        stable &= (rp["id"] == base["id"]) & (rm["id"] == base["id"])
    return fd, stable, t0

# --------------------------------------------------------------------------
# Sec. V: render-accelerated point-to-plane ICP
# --------------------------------------------------------------------------
#
# Sequential depth-image alignment (Sec. V-B): downsample a depth image by 2
# and drop far points; estimate its normals by Eq. (2); render its mesh, each
# pixel carrying the normal of the surface it sees; associate every return of
# the next depth image with the rendered surface at the same pixel when their
# depths differ by less than a tolerance (projective correspondence, Sec. V);
# minimize the point-to-plane error of the associated pairs over the pose.
#
# Readings (the text is silent or garbled on these):
#   * downsampling keeps every second pixel of every second row; a pixel
#     that is not a finite positive depth up to z_max becomes NaN;
#   * Gaussian smoothing renormalizes the weights over the valid pixels of
#     the (2R+1)^2 window; an invalid centre stays NaN;
#   * Eq. (2) takes the tangents (dx, 0, dz_x) and (0, dy, dz_y) with the
#     central differences dz_x = z~(u+1, v) - z~(u-1, v), dz_y alike, and the
#     metric steps dx = 2 z~/fx, dy = 2 z~/fy at the centre, so
#     N = (0, dy, dz_y) x (dx, 0, dz_x) = (dy dz_x, dx dz_y, -dx dy), then
#     normalized (camera frame; it faces the camera, N_z < 0);
#   * a rendered pixel carries the normalized sum of its winning triangle's
#     three vertex normals (flat over the triangle), turned towards the
#     camera; triangles of class FU (skirts at discontinuities and at the
#     range limit) are not surfaces to align to;
#   * the cost of Sec. V step 5, C = sum |Z_M - Z_1|, is summed over the
#     associated pixels.

def downsample(depth, factor=2, z_max=8.0):
    """Every ``factor``-th pixel of every ``factor``-th row; NaN where the
    depth is not finite, not positive or beyond ``z_max``."""
    d = np.asarray(depth, np.float32)[::factor, ::factor].copy()
    with np.errstate(invalid="ignore"):
        bad = ~(np.isfinite(d) & (d > 0) & (d <= np.float32(z_max)))
    d[bad] = np.nan
    return d


def downsample_camera(cam, factor=2):
    """Intrinsics of the downsampled image: pixel (u', v') is (factor u', factor v')."""
    from dataclasses import replace
    H = -(-cam.height // factor)
    W = -(-cam.width // factor)
    return replace(cam, fx=cam.fx / factor, fy=cam.fy / factor, cx=cam.cx / factor, cy=cam.cy / factor,
                   width=W, height=H)


def gaussian_weights(sigma, radius):
    """1-D Gaussian weights over offsets -radius..radius, summing to 1."""
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def smooth_depth(depth, sigma=1.0, radius=2):
    """Gaussian smoothing of a depth image over its valid pixels: at a valid
    centre, sum w_i w_j z / sum w_i w_j over the valid pixels of the window."""
    z = np.asarray(depth, np.float64)
    H, W = z.shape
    w = gaussian_weights(sigma, radius)
    num = np.zeros((H, W)); den = np.zeros((H, W))
    valid = np.isfinite(z)
    zp = np.pad(np.where(valid, z, 0.0), radius)
    vp = np.pad(valid.astype(np.float64), radius)
    for i in range(2 * radius + 1):
        for j in range(2 * radius + 1):
            wij = w[i] * w[j]
            num += wij * zp[i:i + H, j:j + W]
            den += wij * vp[i:i + H, j:j + W]
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(valid, num / den, np.nan)


def depth_normals(depth, cam, sigma=1.0, radius=2):
    """Camera-frame unit normals [H,W,3] of a depth image by Eq. (2) (see the
    readings above); NaN at the border and where the centre or one of its
    four difference neighbours is invalid."""
    zs = smooth_depth(depth, sigma, radius)
    H, W = zs.shape
    N = np.full((H, W, 3), np.nan)
    c = zs[1:-1, 1:-1]
    dzx = zs[1:-1, 2:] - zs[1:-1, :-2]
    dzy = zs[2:, 1:-1] - zs[:-2, 1:-1]
    dx = 2.0 * c / np.float64(np.float32(cam.fx))
    dy = 2.0 * c / np.float64(np.float32(cam.fy))
    n = np.stack([dy * dzx, dx * dzy, -dx * dy], -1)
    with np.errstate(invalid="ignore", divide="ignore"):
        n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    N[1:-1, 1:-1] = n
    return N


def vertex_normals(normals, stride, T_wc):
    """World-frame normal of each meshify node (row-major over the node grid):
    the normal image at the node's pixel (i stride, j stride), rotated by the
    view's rotation.  NaN where the normal is undefined."""
    n = np.asarray(normals, np.float64)[::stride, ::stride].reshape(-1, 3)
    R = np.asarray(T_wc, np.float64).reshape(3, 4)[:, :3]
    return n @ R.T


def icp_terms(rend, mesh, vnormals, scan_d, scan_c, cam, T_wc, tol):
    """Per-pixel projective association and point-to-plane terms.

    A pixel is associated when the scan has a return there (class FO), the
    pixel sees a map FO triangle whose three vertex normals are defined, and
    |z_M - z_1| < tol for the rendered depth z_M and the scan depth z_1.
    With n the camera-frame model normal turned towards the camera and
    ray r: e = n . (P_1 - P_M) = (z_1 - z_M) (n . r), J = [n ; P_1 x n]
    (the derivative under T_wc exp(delta) with the correspondence held)."""
    pix = rend["pixels"]
    ids = rend["id"]
    hit = ids >= 0
    tri = np.asarray(mesh[1])
    cls = np.asarray(mesh[2])
    idc = np.maximum(ids, 0)
    vn = np.asarray(vnormals, np.float64)
    s = vn[tri[idc, 0]] + vn[tri[idc, 1]] + vn[tri[idc, 2]]
    R = np.asarray(T_wc, np.float64).reshape(3, 4)[:, :3]
    nc = s @ R                                  # R^T s, row-wise
    with np.errstate(invalid="ignore", divide="ignore"):
        nc = nc / np.linalg.norm(nc, axis=-1, keepdims=True)
    ray = rays(cam, pix)
    ndr = (nc * ray).sum(-1)
    nc = np.where((ndr < 0)[:, None], nc, -nc)
    ndr = -np.abs(ndr)
    z1 = np.asarray(scan_d, np.float64).reshape(-1)[pix]
    c1 = np.asarray(scan_c).reshape(-1)[pix]
    zM = rend["z"]
    scan_pt = c1 == FO
    model = scan_pt & hit & (cls[idc] == FO) & np.all(np.isfinite(nc), -1)
    with np.errstate(invalid="ignore"):
        dz = zM - z1
        assoc = model & (np.abs(dz) < tol)
    e = np.where(assoc, (z1 - np.where(assoc, zM, 0.0)) * ndr, 0.0)
    P1 = np.where(assoc, z1, 0.0)[:, None] * ray
    J = np.concatenate([nc, np.cross(P1, nc)], -1)
    J = np.where(assoc[:, None], J, 0.0)
    return dict(assoc=assoc, scan_pt=scan_pt, model=model, e=e, J=J, dz=dz, z1=z1, zM=zM, n=nc,
                ray_norm=np.linalg.norm(ray, axis=-1))


def icp_reduce(terms, mask=None):
    """C = sum |z_M - z_1|, sum e^2, counts, b = sum e J, H = sum J^T J."""
    m = np.ones(terms["e"].shape, bool) if mask is None else np.asarray(mask, bool)
    a = terms["assoc"] & m
    e = terms["e"][a]
    J = terms["J"][a]
    return dict(cost=float(np.abs(terms["dz"][a]).sum()), sse=float((e * e).sum()),
                n_scan=int((terms["scan_pt"] & m).sum()), n_model=int((terms["model"] & m).sum()),
                n_assoc=int(a.sum()), jtr=(e[:, None] * J).sum(0), jtj=J.T @ J,
                grad=2.0 * (e[:, None] * J).sum(0))


def icp_step(mesh, vnormals, cam, T_wc, scan_d, scan_c, tol, pixels=None, mode="contract"):
    """One render, association and reduction of the point-to-plane ICP."""
    rend = render(mesh, cam, T_wc, pixels, mode)
    terms = icp_terms(rend, mesh, vnormals, scan_d, scan_c, cam, T_wc, tol)
    out = icp_reduce(terms)
    out["terms"] = terms
    out["render"] = rend
    return out


def icp_tol_ties(terms, tol):
    """Pixels whose association decision lies within the depth tolerance of tol."""
    with np.errstate(invalid="ignore"):
        scale = DEPTH_REL * np.fmax(np.abs(terms["zM"]), np.abs(terms["z1"]))
        return terms["model"] & (np.abs(np.abs(terms["dz"]) - tol) <= scale)


# --------------------------------------------------------------------------
# Reweighted Table I (Sec. IV-C suggests adjusting the weights of the
# penalties and rewards per classification)
# --------------------------------------------------------------------------

TABLE_WEIGHTS = np.array([-1.0, 1.0, -1.0, 1.0, -1.0, 1.0, 0.0, 0.0, 0.0])   # the values printed in Table I


def table_cost_weighted(terms, weights, mask=None):
    """sum over pixels of the weight of the pixel's Table I cell."""
    m = np.ones(terms["cell"].shape, bool) if mask is None else np.asarray(mask, bool)
    return float(np.asarray(weights, np.float64)[terms["cell"][m]].sum())


# --------------------------------------------------------------------------
# Color term.  Sec. IV names color as information a render-based cost takes
# in easily, and Sec. IV-C proposes costs and rewards from the colors of
# corresponding pixels; neither gives a form.  Reading: a pixel corresponds
# when Table I rewards it as FO/FO (both see an occupied surface, depths
# within eps); the map's color there is the intensity of the triangle the
# pixel sees (flat over the triangle, as a per-face colored render shows it);
# a corresponding pixel with both intensities finite is rewarded (-1) when
# they differ by at most tol and penalized (+1) otherwise, like Table I's
# cells.  The difference and the comparison are float32 operations on the
# float32 inputs, as the rasterizer takes them.
# --------------------------------------------------------------------------

COLOR_NONE, COLOR_REWARD, COLOR_PENALTY = -1, 0, 1


def color_cells(terms, rend, tri_color, scan_color, tol):
    """Per-pixel color cell: COLOR_REWARD, COLOR_PENALTY or COLOR_NONE."""
    pix = rend["pixels"]
    ids = rend["id"]
    hit = ids >= 0
    c_m = np.where(hit, np.asarray(tri_color, np.float32)[np.maximum(ids, 0)], np.float32(np.nan))
    c_s = np.asarray(scan_color, np.float32).reshape(-1)[pix]
    out = np.full(pix.shape, COLOR_NONE, np.int64)
    with np.errstate(invalid="ignore"):
        diff = np.abs(c_m.astype(np.float32) - c_s)                  # float32 subtraction
        corr = (terms["cell"] == 0) & np.isfinite(c_m) & np.isfinite(c_s)
        out[corr] = np.where(diff[corr] <= np.float32(tol), COLOR_REWARD, COLOR_PENALTY)
    return out


def color_counts(cells, mask=None):
    """(rewarded, penalized) corresponding pixels."""
    m = np.ones(cells.shape, bool) if mask is None else np.asarray(mask, bool)
    return int((cells[m] == COLOR_REWARD).sum()), int((cells[m] == COLOR_PENALTY).sum())


def table_color_cost_weighted(terms, cells, weights, mask=None):
    """Reweighted Table I plus the color cells: weights[0:9] per Table I cell,
    weights[9] per rewarded and weights[10] per penalized corresponding pixel."""
    w = np.asarray(weights, np.float64)
    nr, npen = color_counts(cells, mask)
    return table_cost_weighted(terms, w[:9], mask) + w[9] * nr + w[10] * npen
