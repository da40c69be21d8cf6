"""Shared helpers of the GPU parity tests: workload maps built with the oracle
(never with the GPU path), pixel samples, and the comparison rules.

Comparison rules (tolerances of the pose-scoring path):
  * triangle ids and coverage: bit-exact except at pixels the oracle flags as
    a depth near-tie (runner-up within 1e-6 relative) or a far-plane tie;
  * depth: within 1e-5 relative, except at grazing pixels (|n^.r^| < 1e-2);
  * E_table and the nine counts: exact over pixels that are not flagged
    (flags above plus Table I threshold ties within the depth tolerance);
  * E_soft, gradient, J^T r, J^T J: within 1e-4 of the L1 mass of the
    per-pixel terms.
"""
from __future__ import annotations

import functools

import numpy as np

from oracle import oracle as O
from workloads import configs

EPS = float(np.float32(0.1))


@functools.lru_cache(maxsize=None)
def workload(name: str):
    return getattr(configs, name)()


@functools.lru_cache(maxsize=None)
def oracle_map(name: str):
    """Map mesh of a workload: procedural, or the union of the oracle's
    meshification of every view."""
    w = workload(name)
    if w.map_mesh is not None:
        return w.map_mesh
    parts = [O.meshify(d, w.cam, T, w.stride, w.z_min, w.z_max, w.max_edge, w.smooth_radius)
             for T, d in zip(w.views, w.view_depths)]
    xyz, tri, cls, off = [], [], [], 0
    for v, t, c in parts:
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
    return np.concatenate(xyz), np.concatenate(tri).astype(np.int32), np.concatenate(cls)


@functools.lru_cache(maxsize=None)
def stream(name: str):
    return getattr(configs, name)()


@functools.lru_cache(maxsize=None)
def stream_map(name: str):
    """Map mesh of a multi-scan stream: the oracle's meshification of every view."""
    st = stream(name)
    parts = [O.meshify(d, st.view_cam, T, st.stride, st.z_min, st.z_max, st.max_edge, st.smooth_radius)
             for T, d in zip(st.views, st.view_depths)]
    xyz, tri, cls, off = [], [], [], 0
    for v, t, c in parts:
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
    return np.concatenate(xyz), np.concatenate(tri).astype(np.int32), np.concatenate(cls)


def sample_pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    N = cam.width * cam.height
    return np.sort(rng.choice(N, size=min(n, N), replace=False)).astype(np.int64)


def render_mismatch(rend, cam, g_depth, g_tri):
    """Returns (n_id_mismatch_unflagged, max_rel_depth_err_unflagged, n_flagged)."""
    pix = rend["pixels"]
    fl = O.flags(rend, cam)
    gid = g_tri.reshape(-1)[pix]
    gz = g_depth.reshape(-1)[pix].astype(np.float64)
    ex = fl["near_tie"] | fl["far_tie"]
    bad = (gid != rend["id"]) & ~ex
    ok = (rend["id"] >= 0) & (gid == rend["id"]) & ~fl["grazing"]
    rel = np.abs(gz[ok] - rend["z"][ok]) / rend["z"][ok] if ok.any() else np.zeros(1)
    return int(bad.sum()), float(rel.max()), int(ex.sum())


def flagged_pixels(rend, terms, cam, eps):
    fl = O.flags(rend, cam)
    return fl["near_tie"] | fl["far_tie"] | fl["grazing"] | O.threshold_ties(terms, eps)


def compare_records(g, ref, terms, mask, eps, grad=True, tol=1e-4):
    """Asserts a GPU result record against the oracle's reduction over `mask`."""
    m = mask
    assert g[0] == ref["e_table"], (g[0], ref["e_table"])
    np.testing.assert_array_equal(g[2:11], ref["counts"])
    l1 = max(np.abs(terms["rho"][m]).sum(), 1.0)
    assert abs(g[1] - ref["e_soft"]) <= tol * l1, (g[1], ref["e_soft"], l1)
    if not grad:
        return
    assert g[11] == ref["n_active"], (g[11], ref["n_active"])
    J = terms["J"][m]; r = terms["r"][m]; act = terms["active"][m]
    b_l1 = np.abs(r[act, None] * J[act]).sum(0)
    H_l1 = np.abs(J[act][:, :, None] * J[act][:, None, :]).sum(0)
    gb = g[18:24]
    assert (np.abs(gb - ref["jtr"]) <= tol * np.maximum(b_l1, 1e-12)).all(), (gb, ref["jtr"], b_l1)
    gg = g[12:18]
    assert (np.abs(gg - (4.0 / eps ** 2) * ref["jtr"]) <= tol * (4.0 / eps ** 2) * np.maximum(b_l1, 1e-12)).all()
    iu = np.triu_indices(6)
    gH = g[24:45]
    assert (np.abs(gH - ref["jtj"][iu]) <= tol * np.maximum(H_l1[iu], 1e-12)).all(), (gH, ref["jtj"][iu])
