"""Benchmark of the pose-scoring hot path on one MI355X.

Workload (the differentiation configuration): a 6 x 5 x 2.8 m synthetic room
with 16 boxes and a doorway, mapped by meshifying 27 simulated 640x480 range
images at stride 4 on the GPU (1,021,734 triangles, free-occupied and
free-unknown); a held-out 640x480 query scan; 64 candidate poses 10 cm / 5 deg
from the truth.  One step = cost + se(3) gradient + Gauss-Newton blocks for
all 64 poses (cluster cull, tile rasterization with the fused Table I /
E_soft / Jacobian resolve, per-pose reduction) followed by the on-device
Levenberg-Marquardt pose update.  Inputs are resident in HBM before timing.

Prints one JSON line.  Timing: W untimed warm-up steps, then K steps between
two device synchronizations; the rasterizer's own launches are timed with
HIP events on their stream over the same region (roofline).  The FP64 oracle
is timed on the host over a bounded pixel sample of one pose (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pose cost+grad evals/s @640x480, 1M-tri mesh; scans aligned/s vs plain form"
HBM_PEAK_GBS = 8000.0
# DRAM bytes of one rasterizer launch from rocprofv3 FETCH_SIZE/WRITE_SIZE,
# scaled by a plain-copy calibration (profiles/k_raster_differentiation.md);
# valid only for the rasterizer source and tile they were taken with (the
# prefix moves with a comment-only edit whose device assembly is unchanged).
PROFILED_TRAFFIC = {"rm_raster_sha256_16": "cf7798a3c4dbfc6a", "tile": [64, 32],
                    # calibrated FETCH_SIZE + WRITE_SIZE of one rasterizer and one
                    # binning launch, and the rasterizer's VALU issue fraction
                    # (profiles/k_raster_differentiation.md)
                    "bytes_per_launch": 1327.2e6, "bin_bytes_per_launch": 1218.2e6, "valu_issue_frac": 0.817,
                    # SQ_INSTS_LDS_ATOMIC_BANDWIDTH x 8: 64-bit LDS atomic lanes of one
                    # rasterizer launch (an upper bound: the few 32-bit queue counters
                    # count as well), and TCC_ATOMIC_sum of one binning launch and its
                    # profiled duration (profiles/atomics_differentiation.md)
                    "lds_atomic_lanes_per_launch": 1.924e8, "bin_global_atomics_per_launch": 7.428e5,
                    "bin_launch_ms": 0.931}


def profiled_traffic(tile, field="bytes_per_launch"):
    """A figure of the committed rocprofv3 summary of the rasterizer, or None
    once the source or the tile differs from the profiled one."""
    import hashlib
    src = os.path.join(ROOT, "paper_1702_06813_amd", "csrc", "rm_raster.hip")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    ok = h == PROFILED_TRAFFIC["rm_raster_sha256_16"] and list(tile) == PROFILED_TRAFFIC["tile"]
    return PROFILED_TRAFFIC[field] if ok else None


def atomic_peaks(sweep=False):
    """Throughput peaks of the LDS 64-bit minimum (the depth-key resolve, per
    lane) and of the global 32-bit add with return (bin reservations), from
    librm_microbench.so; None where that library was not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_1702_06813_amd", "librm_microbench.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.rm_mb_lds_min_u64.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    lib.rm_mb_global_atomic_add.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    lib.rm_mb_lds_min_u64.restype = lib.rm_mb_global_atomic_add.restype = ctypes.c_int
    sec, ops = ctypes.c_double(), ctypes.c_double()

    def rate(rc):
        return ops.value / sec.value if rc == 0 and sec.value > 0 else None

    lds, glob = {}, {}
    for blocks in ((1024, 2048, 4096) if sweep else (2048,)):
        lds[blocks] = rate(lib.rm_mb_lds_min_u64(blocks, 8192, ctypes.byref(sec), ctypes.byref(ops)))
    for slots_log2 in ((12, 15, 20) if sweep else (15,)):
        glob[slots_log2] = rate(lib.rm_mb_global_atomic_add(2048, 256, slots_log2, ctypes.byref(sec),
                                                            ctypes.byref(ops)))
    best = lambda d: max((v for v in d.values() if v), default=None)
    out = {"lds_min_u64_lane_ops_per_s": best(lds), "global_atomic_add_per_s": best(glob)}
    if sweep:
        out["lds_by_blocks"] = lds
        out["global_by_slots_log2"] = glob
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(rm, torch, dev):
    from workloads import configs
    t0 = time.time()
    w = configs.differentiation()
    log(f"workload generated in {time.time() - t0:.1f}s")
    parts = [rm.mesh_from_range(torch.from_numpy(d).to(dev), w.cam, T, w.stride, w.z_min, w.z_max, w.max_edge,
                               w.smooth_radius)
             for T, d in zip(w.views, w.view_depths)]
    mesh = rm.Mesh.concat(parts).prepare()
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(dev), w.z_min, w.z_max, cam=w.cam)
    T0 = torch.from_numpy(np.ascontiguousarray(w.poses.reshape(-1, 12))).to(dev)
    torch.cuda.synchronize()
    log(f"map: {mesh.n_tris} triangles, {mesh.xyz.shape[0]} vertices; {T0.shape[0]} poses")
    return w, mesh, scan, T0


def cpu_baseline(w, torch, n_poses=2):
    """FP64 oracle: cost + gradient of the first poses, full frame, on the
    host's cores (no extrapolation)."""
    from oracle import oracle as O
    O.build()
    off = 0
    xyz, tri, cls = [], [], []
    for T, d in zip(w.views, w.view_depths):
        v, t, c = O.meshify(d, w.cam, T, w.stride, w.z_min, w.z_max, w.max_edge, w.smooth_radius)
        xyz.append(v); tri.append(t + off); cls.append(c); off += len(v)
    mesh_np = (np.concatenate(xyz), np.concatenate(tri).astype(np.int32), np.concatenate(cls))
    d, c = O.scan_image(w.scan_depth, w.z_min, w.z_max)
    t0 = time.perf_counter()
    for k in range(n_poses):
        O.align_cost(mesh_np, w.cam, w.poses[k], d, c, eps=0.1)
    t = time.perf_counter() - t0
    return {"value": n_poses / t, "unit": "pose-evals/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{n_poses} of the 64 poses, full 640x480 frame each, against the 1,021,734-triangle map "
                      f"({t:.1f} s wall)"}


def alignment_comparison(rm, torch, w, mesh, scan, T0, n_plain=16, reps=3):
    """Scans aligned per second on the differentiation workload, each from
    the same 10 cm / 5 deg starts, with final pose errors:
      * the batched gradient forms: all 64 starts in one launch per
        iteration, 20 iterations with the eps schedule, replayed from one
        captured hipGraph, Gauss-Newton (LM) and Adam;
      * the paper's plain form (one pose per launch, cost only, the
        derivative-free hybrid optimizer, up to 700 evaluations) on n_plain
        starts, and the same optimizer with the independent points of one
        alignment evaluated together (same poses, fewer launches);
      * the paper's optimizer for all 64 starts in lockstep (one launch per
        round of evaluations over every start; the starts already fill the
        launch, so speculative batches would only add evaluations);
      * the ablation of the gradient form with one pose per launch, no graph
        and one workgroup per item (no persistent scheduling);
      * the batched GN alignment against the map meshed without node
        smoothing (radius 0), to show what that reading of the paper's
        suggested blurring buys."""
    from paper_1702_06813_amd import align as A
    B = T0.shape[0]
    res = {}
    d0, a0 = A.pose_errors(w.poses, w.T_true)
    res["initial_error_m_median"] = float(np.median(d0))
    res["initial_error_deg_median"] = float(np.degrees(np.median(a0)))
    for method in ("gn", "adam"):
        al = A.BatchedAligner(mesh, scan, B, iters=20, method=method)
        al.run(T0, use_graph=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            Tb = al.run(T0, use_graph=True)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        dtb, dab = A.pose_errors(Tb.cpu().numpy(), w.T_true)
        log(f"batched {method}: {B} scans in {tb * 1e3:.1f} ms; median error {np.median(dtb) * 100:.2f} cm "
            f"{np.degrees(np.median(dab)):.3f} deg")
        key = "batched" if method == "gn" else "batched_adam"
        res[f"{key}_scans_per_s"] = B / tb
        res[f"{key}_error_m_median"] = float(np.median(dtb))
        res[f"{key}_error_deg_median"] = float(np.degrees(np.median(dab)))
        if method == "gn":
            res["batched_error_m_same_starts"] = float(np.median(dtb[:n_plain]))
            res["batched_error_deg_same_starts"] = float(np.degrees(np.median(dab[:n_plain])))
            tgn, dtb_gn = tb, dtb
    res["iterations"] = 20
    # the paper's plain form, one evaluation per launch, and batched within each alignment
    for form in ("plain", "plain_within"):
        Tp, evs, nl = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_plain):
            if form == "plain":
                T, e, ev = A.plain_align(mesh, scan, w.poses[k], eps=0.1, budget=700)
                nl.append(ev)
            else:
                T, e, ev, launches = A.plain_align_batched(mesh, scan, w.poses[k], eps=0.1, budget=700)
                nl.append(launches)
            Tp.append(T); evs.append(ev)
        tp = (time.perf_counter() - t0) / n_plain
        dtp, dap = A.pose_errors(np.stack(Tp), w.T_true)
        log(f"{form}: {n_plain} scans, {tp * 1e3:.1f} ms each, {np.mean(nl):.0f} launches each; median error "
            f"{np.median(dtp) * 100:.2f} cm {np.degrees(np.median(dap)):.3f} deg")
        res[f"{form}_scans_per_s"] = 1.0 / tp
        res[f"{form}_launches_mean"] = float(np.mean(nl))
        res[f"{form}_evaluations_mean"] = float(np.mean(evs))
        res[f"{form}_error_m_median"] = float(np.median(dtp))
        res[f"{form}_error_deg_median"] = float(np.degrees(np.median(dap)))
        if form == "plain":
            tplain = tp
    res["n_plain_scans"] = n_plain
    res["speedup_vs_plain"] = tplain * B / tgn
    # the paper's optimizer for all B starts in lockstep, speculative batches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Tq, _, evq, launches = A.batched_plain_align(mesh, scan, w.poses, eps=0.1, budget=700)
    tq = time.perf_counter() - t0
    dtq, daq = A.pose_errors(Tq, w.T_true)
    log(f"batched plain form: {B} scans in {tq:.2f} s ({launches} launches); median error "
        f"{np.median(dtq) * 100:.2f} cm {np.degrees(np.median(daq)):.3f} deg")
    res.update({"batched_plain_form_scans_per_s": B / tq, "batched_plain_form_launches": int(launches),
                "batched_plain_form_error_m_median": float(np.median(dtq)),
                "batched_plain_form_error_deg_median": float(np.degrees(np.median(daq)))})
    # ablation: the gradient form with one pose per launch, eager, one workgroup per item
    ctx = rm.context(T0.device)
    ctx.set_schedule(1)
    try:
        n_abl = 8
        al1 = A.BatchedAligner(mesh, scan, 1, iters=20)
        al1.run(T0[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ta = [al1.run(T0[k:k + 1]).clone() for k in range(n_abl)]
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / n_abl
    finally:
        ctx.set_schedule(0)
    dta, daa = A.pose_errors(torch.cat(Ta).cpu().numpy(), w.T_true)
    log(f"one pose per launch (gradient, eager): {ta * 1e3:.1f} ms per scan; median error "
        f"{np.median(dta) * 100:.2f} cm")
    res.update({"one_pose_per_launch_grad_scans_per_s": 1.0 / ta,
                "one_pose_per_launch_grad_error_m_median": float(np.median(dta)),
                "batched_vs_one_pose_per_launch": ta * B / tgn})
    # what the node smoothing of the map meshing buys: the same batched GN
    # alignment against the map meshed without it (smoothing radius 0)
    parts = [rm.mesh_from_range(torch.from_numpy(d).to(T0.device), w.cam, T, w.stride, w.z_min, w.z_max,
                                w.max_edge, 0) for T, d in zip(w.views, w.view_depths)]
    mesh0 = rm.Mesh.concat(parts).prepare()
    T0b = A.BatchedAligner(mesh0, scan, B, iters=20).run(T0, use_graph=False)
    dt0, da0 = A.pose_errors(T0b.cpu().numpy(), w.T_true)
    log(f"batched gn, map meshed without smoothing: median error {np.median(dt0) * 100:.2f} cm "
        f"{np.degrees(np.median(da0)):.3f} deg, {int((dt0 < 0.02).sum())}/{B} under 2 cm")
    res.update({"unsmoothed_map_batched_error_m_median": float(np.median(dt0)),
                "unsmoothed_map_batched_error_deg_median": float(np.degrees(np.median(da0))),
                "unsmoothed_map_under_2cm": int((dt0 < 0.02).sum()),
                "smoothed_map_under_2cm": int((dtb_gn < 0.02).sum())})
    return res


def config_throughput(rm, torch, dev, name, steps=10):
    """Pose-evals/s of one more workload: tiny (64x48, ~2.4k triangles, one
    pose, cost only), kinect (640x480, ~186k triangles, 64 poses, cost only)
    or wide (1280x960, ~4M triangles, 256 poses, cost + gradient, tile
    autotuned).  Inputs resident before timing; W = 3 warm-up calls (the
    first sizes the bins, and for wide runs the autotuner)."""
    from workloads import configs
    t0 = time.time()
    w = getattr(configs, name)()
    if w.map_mesh is not None:
        mesh = rm.Mesh.from_arrays(*w.map_mesh, device=dev).prepare()
    else:
        parts = [rm.mesh_from_range(torch.from_numpy(d).to(dev), w.cam, T, w.stride, w.z_min, w.z_max, w.max_edge,
                                    w.smooth_radius) for T, d in zip(w.views, w.view_depths)]
        mesh = rm.Mesh.concat(parts).prepare()
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(dev), w.z_min, w.z_max, cam=w.cam)
    T = torch.from_numpy(np.ascontiguousarray(w.poses.reshape(-1, 12))).to(dev)
    grad = name == "wide"
    f = rm.align_cost_grad if grad else rm.align_cost
    ctx = rm.context(dev)
    ctx.autotune(name == "wide")
    out = torch.empty((T.shape[0], rm.OUT_STRIDE), dtype=torch.float64, device=dev)
    try:
        for _ in range(3):
            f(mesh, scan, T, 0.1, out=out)
        torch.cuda.synchronize()
        ctx.profile(True); ctx.profile_read()
        t1 = time.perf_counter()
        for _ in range(steps):
            f(mesh, scan, T, 0.1, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        n, ms = ctx.profile_read()
    finally:
        ctx.profile(False)
        ctx.autotune(False)
    tile = ctx.get_tile(w.cam.width, w.cam.height, T.shape[0], mesh.n_tris)
    log(f"{name}: {T.shape[0]} poses, {mesh.n_tris} triangles, {w.cam.width}x{w.cam.height}: {dt * 1e3:.3f} ms per "
        f"call, {T.shape[0] / dt:.0f} pose-evals/s (tile {tile}, set up in {time.time() - t0:.1f}s)")
    return {"pose_evals_per_s": T.shape[0] / dt, "ms_per_call": dt * 1e3, "raster_ms": ms / max(n, 1),
            "poses": int(T.shape[0]), "n_tris": int(mesh.n_tris), "image": [w.cam.width, w.cam.height],
            "mode": "cost + gradient" if grad else "cost", "tile": list(tile), "autotuned": name == "wide"}


def uneven_stream(rm, torch, dev, steps=5):
    """Pose-evals/s of the uneven stream: 32 scans cycling 320x240, 640x480
    and 1280x960 with 16-128 candidates each (2,522 poses) against the
    2.1M-triangle corridor map, cost + gradient in one launch.  Its 712,110
    (pose, tile) records are too many for bins holding its fullest tile in
    the memory budget, so this is the workload of the bin overflow (spill
    list and exact regions).  W = 3 warm-up calls (the first sizes bins and
    overflow)."""
    from workloads import configs
    t0 = time.time()
    st = configs.uneven()
    parts = [rm.mesh_from_range(torch.from_numpy(d).to(dev), st.view_cam, T, st.stride, st.z_min, st.z_max,
                                st.max_edge, st.smooth_radius) for T, d in zip(st.views, st.view_depths)]
    mesh = rm.Mesh.concat(parts).prepare()
    scans = [rm.scan_image(torch.from_numpy(x.depth).to(dev), st.z_min, st.z_max, cam=x.cam) for x in st.scans]
    counts = [len(x.poses) for x in st.scans]
    T = torch.from_numpy(np.ascontiguousarray(np.concatenate([x.poses for x in st.scans]).reshape(-1, 12))).to(dev)
    out = torch.empty((T.shape[0], rm.OUT_STRIDE), dtype=torch.float64, device=dev)
    ctx = rm.context(dev)
    try:
        for _ in range(3):
            rm.align_cost_grad(mesh, scans, T, 0.1, poses_per_scan=counts, out=out)
        torch.cuda.synchronize()
        ctx.profile(True); ctx.profile_read(); ctx.profile_read_binning()
        t1 = time.perf_counter()
        for _ in range(steps):
            rm.align_cost_grad(mesh, scans, T, 0.1, poses_per_scan=counts, out=out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        n, ms = ctx.profile_read()
        nb, bms = ctx.profile_read_binning()
    finally:
        ctx.profile(False)
    log(f"uneven stream: {T.shape[0]} poses in {len(scans)} scans, {mesh.n_tris} triangles: {dt * 1e3:.1f} ms per "
        f"call ({ms / max(n, 1):.1f} rasterizing, {bms / max(nb, 1):.1f} binning), {T.shape[0] / dt:.0f} "
        f"pose-evals/s (set up in {time.time() - t0:.1f}s)")
    return {"pose_evals_per_s": T.shape[0] / dt, "ms_per_call": dt * 1e3, "raster_ms": ms / max(n, 1),
            "bin_ms": bms / max(nb, 1), "poses": int(T.shape[0]), "scans": len(scans), "n_tris": int(mesh.n_tris),
            "mode": "cost + gradient"}


def trajectory_c5(rm, torch, dev, n_scans=500):
    """Scan-to-map alignment of a 500-scan looped walk (0.5 m/s at 2 Hz, 0.25
    m apart) around an 8 x 6 m office room with 24 boxes, scans cycling
    320x240, 640x480 and 1280x960, against the ~2.2M-triangle map of 130
    meshified views:
    every scan from exactly 10 cm / 5 deg off its truth, 20 Gauss-Newton
    iterations, 32 scans per launch, one captured graph per batch shape.
    Timed: the whole alignment of all scans (staging copies, graph replays,
    pose read-back); not timed: generation, meshing, the warm-up pass.  Beside
    it, the paper's plain form (one pose per launch, cost only) on the first
    12 scans of the walk, for scans/s and errors on different scans."""
    from paper_1702_06813_amd import align as A
    from workloads import configs
    t0 = time.time()
    tr = configs.trajectory(n_scans=n_scans)
    parts = [rm.mesh_from_range(torch.from_numpy(d).to(dev), tr.view_cam, T, tr.stride, tr.z_min, tr.z_max,
                                tr.max_edge, tr.smooth_radius) for T, d in zip(tr.views, tr.view_depths)]
    mesh = rm.Mesh.concat(parts).prepare()
    scans = [rm.scan_image(torch.from_numpy(s.depth).to(dev), tr.z_min, tr.z_max, cam=s.cam) for s in tr.scans]
    T0 = np.stack([s.poses[0] for s in tr.scans])
    truth = np.stack([s.T_true for s in tr.scans])
    torch.cuda.synchronize()
    log(f"trajectory: {len(scans)} scans, map {mesh.n_tris} triangles, set up in {time.time() - t0:.1f}s")
    ta = A.TrajectoryAligner(mesh)
    ta.run(scans, T0)                                  # sizes scratch and captures the graphs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T, launches = ta.run(scans, T0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    errs = [A.pose_errors(T[j], truth[j]) for j in range(len(T))]
    dt_m = np.array([e[0][0] for e in errs]); da = np.degrees(np.array([e[1][0] for e in errs]))
    d0 = np.array([A.pose_errors(T0[j], truth[j])[0][0] for j in range(len(T))])
    log(f"trajectory: {len(T) / dt:.0f} scans/s ({launches} cost launches, {len(ta.shapes)} graph shapes); RMSE "
        f"{np.sqrt(np.mean(dt_m ** 2)) * 100:.2f} cm {np.sqrt(np.mean(da ** 2)):.3f} deg (initial "
        f"{np.sqrt(np.mean(d0 ** 2)) * 100:.1f} cm)")
    # the paper's plain form on different scans of the walk: the first n_plain
    # scans (all three resolutions), one pose per launch, cost only
    n_plain = 12
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Tp = [A.plain_align(mesh, scans[j], T0[j], eps=0.1, budget=700)[0] for j in range(n_plain)]
    tp = (time.perf_counter() - t1) / n_plain
    dpl = np.array([A.pose_errors(Tp[j], truth[j])[0][0] for j in range(n_plain)])
    log(f"trajectory, plain form on {n_plain} scans: {1.0 / tp:.2f} scans/s, median {np.median(dpl) * 100:.2f} cm "
        f"(batched on the same scans: median {np.median(dt_m[:n_plain]) * 100:.2f} cm)")
    return {"scans": len(T), "scans_per_s": len(T) / dt, "wall_s": dt, "cost_launches": int(launches),
            "graph_shapes": len(ta.shapes), "map_tris": int(mesh.n_tris),
            "rmse_m": float(np.sqrt(np.mean(dt_m ** 2))), "rmse_deg": float(np.sqrt(np.mean(da ** 2))),
            "median_error_m": float(np.median(dt_m)), "p90_error_m": float(np.percentile(dt_m, 90)),
            "scans_over_5cm": int((dt_m > 0.05).sum()),
            "initial_rmse_m": float(np.sqrt(np.mean(d0 ** 2))),
            "plain_form_scans": n_plain, "plain_form_scans_per_s": 1.0 / tp,
            "plain_form_error_m_median": float(np.median(dpl)),
            "batched_error_m_median_same_scans": float(np.median(dt_m[:n_plain])),
            "speedup_vs_plain_form": (len(T) / dt) * tp,
            "paper_context": "the paper aligns scans one second apart at about 2 Hz on a GTX 765M"}


def color_term(rm, torch, dev, w, mesh, scan, T0, steps=20):
    """The color term (Sec. IV, IV-C).
      * throughput: the benchmarked step (64 poses, cost + gradient + LM
        update) on the 1M-triangle map with and without colors (triangle
        albedo at the centroids, the scan's intensity image);
      * textured wall: the paper's derivative-free optimizer (speculative
        batches within each alignment) from 8 starts N(0, 4 cm) / N(0, 1.5
        deg) per axis, on E(X) alone and on E(X) + color counts (weights -1 /
        +1, tol 0.02), with the final errors per direction of the camera
        frame: depth alone fixes none of the in-plane motion."""
    from paper_1702_06813_amd import align as A
    from workloads import configs, scenes as S
    xyz = mesh.xyz.cpu().numpy(); tri = mesh.tri.cpu().numpy()
    cmesh = rm.Mesh(mesh.xyz, mesh.tri, mesh.cls, mesh.clusters,
                    torch.from_numpy(S.triangle_albedo(xyz, tri)).to(dev))
    cscan = rm.Scan(scan.depth, scan.cls, scan.cam,
                    color=torch.from_numpy(S.intensity_image(w.scene, w.cam, w.T_true, 91, noise=0.02)).to(dev))
    B = T0.shape[0]
    out = torch.empty((B, rm.OUT_STRIDE), dtype=torch.float64, device=dev)
    res = {}
    for key, m_, s_ in (("without_color", mesh, scan), ("with_color", cmesh, cscan)):
        T = T0.clone()
        for _ in range(3):
            rm.align_cost_grad(m_, s_, T, 0.1, out=out, color_tol=0.05)
            rm.gn_step(out, T, 1e-3)
        T.copy_(T0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            rm.align_cost_grad(m_, s_, T, 0.1, out=out, color_tol=0.05)
            rm.gn_step(out, T, 1e-3)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / steps
        res[key] = {"ms_per_step": dt * 1e3, "pose_evals_per_s": B / dt}
    o = out.cpu().numpy()
    res["with_color"]["corresponding_px_per_pose"] = float(
        (o[:, rm.OUT_COLOR_REWARD] + o[:, rm.OUT_COLOR_PENALTY]).mean())
    res["overhead"] = res["with_color"]["ms_per_step"] / res["without_color"]["ms_per_step"] - 1.0
    log(f"color: step {res['without_color']['ms_per_step']:.3f} ms without, "
        f"{res['with_color']['ms_per_step']:.3f} ms with colors")

    wl = configs.textured_wall()
    wm = rm.Mesh.from_arrays(*wl.map_mesh, device=dev)
    wm.color = torch.from_numpy(wl.map_color).to(dev)
    wm.prepare()
    ws = rm.scan_image(torch.from_numpy(wl.scan_depth).to(dev), wl.z_min, wl.z_max, cam=wl.cam)
    ws.color = torch.from_numpy(wl.scan_color).to(dev)
    wts = list(rm.TABLE_WEIGHTS) + [-1.0, 1.0]
    tol = 0.02
    Rt = wl.T_true[:, :3]

    def directions(Tp):
        # camera-frame error components: in-plane (x, y) and along the axis,
        # rotation about the axis (roll) and across it (pan / tilt)
        d = Rt.T @ (Tp[:, 3] - wl.T_true[:, 3])
        Rr = Rt.T @ Tp[:, :3]
        rv = np.array([Rr[2, 1] - Rr[1, 2], Rr[0, 2] - Rr[2, 0], Rr[1, 0] - Rr[0, 1]]) / 2
        return np.hypot(d[0], d[1]), abs(d[2]), np.degrees(abs(rv[2])), np.degrees(np.hypot(rv[0], rv[1]))

    def summary(poses):
        e = np.array([directions(Tp) for Tp in poses])
        return {"in_plane_m_median": float(np.median(e[:, 0])), "depth_m_median": float(np.median(e[:, 1])),
                "roll_deg_median": float(np.median(e[:, 2])), "tilt_deg_median": float(np.median(e[:, 3]))}

    A.plain_align_batched(wm, ws, wl.poses[0], budget=50, weights=wts, color_tol=tol)     # warm-up
    wall = {"initial": summary(wl.poses)}
    for key, weights in (("depth_only", None), ("depth_and_color", wts)):
        t1 = time.perf_counter()
        runs = [A.plain_align_batched(wm, ws, Tp, weights=weights, color_tol=tol) for Tp in wl.poses]
        dt = time.perf_counter() - t1
        wall[key] = summary([r[0] for r in runs])
        wall[key].update({"scans_per_s": len(runs) / dt, "launches_mean": float(np.mean([r[3] for r in runs])),
                          "evaluations_mean": float(np.mean([r[2] for r in runs]))})
        log(f"color wall {key}: in-plane {wall[key]['in_plane_m_median'] * 100:.2f} cm, depth "
            f"{wall[key]['depth_m_median'] * 100:.2f} cm, roll {wall[key]['roll_deg_median']:.3f} deg, tilt "
            f"{wall[key]['tilt_deg_median']:.3f} deg; {len(runs) / dt:.1f} scans/s")
    wall.update({"starts": len(wl.poses), "color_tol": tol, "color_weights": [-1.0, 1.0], "eps": 0.1,
                 "n_tris": int(wm.n_tris), "image": [wl.cam.width, wl.cam.height]})
    res["textured_wall"] = wall
    return res


def icp_odometry(rm, torch, dev, n_frames=33, iters=10, reps=3):
    """Sequential depth-image alignment (Sec. V-B) on a 33-frame Kinect-like
    sequence (32 consecutive pairs, ~3.5 cm / 1.5 deg apart, 320x240 after
    downsampling): the preparation of every pair (downsampling, Eq. (2)
    normals, meshing, vertex normals) and `iters` ICP iterations for all 32
    pairs in one launch each, from the identity start; errors against the
    sequence's ground truth."""
    from paper_1702_06813_amd import align as A
    from workloads import configs
    seq = configs.odometry(n_frames=n_frames)
    depths = [torch.from_numpy(d).to(dev) for d in seq.depths]
    ks = list(range(n_frames - 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh, vn, scans, offs, cam2 = A.prepare_pairs(depths, seq.cam, ks)
    torch.cuda.synchronize()
    tprep = time.perf_counter() - t0
    T0 = torch.from_numpy(np.ascontiguousarray(offs.reshape(-1, 12))).to(dev)
    pps = [1] * len(ks)
    A.icp_align(mesh, vn, scans, T0, 0.1, iters, 1e-6, pps)       # first call of the shape: tile autotune
    ctx = rm.context(dev)
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        T, out = A.icp_align(mesh, vn, scans, T0, 0.1, iters, 1e-6, pps)
    torch.cuda.synchronize()
    ticp = (time.perf_counter() - t0) / reps
    n, ms = ctx.profile_read()
    ctx.profile(False)
    Tn = T.cpu().numpy()
    dts, das = [], []
    for j, k in enumerate(ks):
        rel = Tn[j].copy()
        rel[:, 3] -= offs[j][:, 3]
        truth = (np.linalg.inv(np.vstack([seq.poses[k], [0, 0, 0, 1]])) @ np.vstack([seq.poses[k + 1], [0, 0, 0, 1]]))[:3]
        dt, da = A.pose_errors(rel[None], truth)
        dts.append(dt[0]); das.append(da[0])
    dts, das = np.array(dts), np.degrees(np.array(das))
    o = out.cpu().numpy()
    log(f"icp odometry: {len(ks)} pairs, prepare {tprep * 1e3:.1f} ms, {iters} iterations {ticp * 1e3:.1f} ms "
        f"({ms / max(n, 1):.3f} ms per raster launch); error median {np.median(dts) * 1e3:.2f} mm "
        f"{np.median(das):.3f} deg, max {dts.max() * 1e3:.2f} mm {das.max():.3f} deg")
    return {"pairs": len(ks), "image": [int(cam2.width), int(cam2.height)], "iterations": iters,
            "model_tris": int(mesh.tri.shape[0]), "prepare_ms": tprep * 1e3, "icp_ms": ticp * 1e3,
            "pairs_per_s": len(ks) / (tprep + ticp), "icp_pairs_per_s": len(ks) / ticp,
            "raster_ms_per_launch": ms / max(n, 1),
            "error_mm_median": float(np.median(dts) * 1e3), "error_mm_max": float(dts.max() * 1e3),
            "error_deg_median": float(np.median(das)), "error_deg_max": float(das.max()),
            "associated_pixels_median": float(np.median(o[:, 11])),
            "motion_mm_median": float(np.median([np.linalg.norm(seq.poses[k + 1][:, 3] - seq.poses[k][:, 3])
                                                 for k in ks]) * 1e3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-alignment", action="store_true", help="skip the batched-vs-plain alignment comparison")
    ap.add_argument("--no-icp", action="store_true", help="skip the render-accelerated ICP odometry (Sec. V)")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' throughput lines")
    ap.add_argument("--configs", default="tiny,kinect,wide,uneven",
                    help="comma-separated workloads for the throughput lines (tiny, kinect, wide, uneven)")
    ap.add_argument("--no-trajectory", action="store_true", help="skip the 500-scan trajectory alignment")
    ap.add_argument("--no-color", action="store_true", help="skip the color term's throughput and wall alignment")
    ap.add_argument("--atomic-peaks", action="store_true",
                    help="only run the atomic-throughput microbenchmarks (a small sweep of launch shapes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the pose-scoring path is built and "
              f"measured on a single MI355X", file=sys.stderr)
        sys.exit(2)
    config_names = [n for n in args.configs.split(",") if n]
    unknown = sorted(set(config_names) - {"tiny", "kinect", "wide", "uneven"})
    if unknown:
        print(f"bench.py: unknown workload(s) in --configs: {', '.join(unknown)} "
              f"(known: tiny, kinect, wide, uneven)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1702_06813_amd as rm

    dev = torch.device("cuda:0")
    if args.atomic_peaks:
        torch.zeros(1, device=dev)
        print(json.dumps(atomic_peaks(sweep=True)), flush=True)
        return
    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)
        return
    w, mesh, scan, T0 = build_inputs(rm, torch, dev)
    B = T0.shape[0]
    eps, lam = 0.1, 1e-3
    T = T0.clone()
    out = torch.empty((B, rm.OUT_STRIDE), dtype=torch.float64, device=dev)
    ctx = rm.context(dev)
    ctx.autotune(True)              # picks the tile shape on the first call of this shape

    def step():
        rm.align_cost_grad(mesh, scan, T, eps, out=out)
        rm.gn_step(out, T, lam)

    for _ in range(args.warmup):
        step()
    T.copy_(T0)
    torch.cuda.synchronize()
    log(f"warm-up done ({args.warmup} steps)")

    ctx.profile(True)
    ctx.profile_read()
    ctx.profile_read_binning()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_launch, raster_ms = ctx.profile_read()
    n_bin, bin_ms = ctx.profile_read_binning()
    ctx.profile(False)
    wall = t1 - t0
    log(f"timed {args.steps} steps in {wall * 1e3:.1f} ms; rasterizer {n_launch} launches, {raster_ms:.2f} ms")

    # algorithmic bytes of one rasterizer launch (B poses): visible mesh, scan image, outputs
    o = out.cpu().numpy()
    t_vis = o[:, rm.OUT_N_VISIBLE]
    v_per_t = mesh.xyz.shape[0] / max(mesh.n_tris, 1)
    W, H = w.cam.width, w.cam.height
    bytes_launch = float(np.sum(12.0 * v_per_t * t_vis + 13.0 * t_vis + 5.0 * W * H + 8 * 3 + 4 * 9 + 4 * 34))
    avg_s = raster_ms / max(n_launch, 1) / 1e3
    achieved = bytes_launch / avg_s / 1e9
    # the binning pass reads the visible mesh once per pose (indices and vertices)
    bin_bytes = float(np.sum(12.0 * v_per_t * t_vis + 12.0 * t_vis))
    bin_s = bin_ms / max(n_bin, 1) / 1e3

    # the same step replayed from one captured hipGraph
    T.copy_(T0)
    step()
    torch.cuda.synchronize()
    g = rm.Graph(dev)
    with g:
        step()
    g.replay()
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - tg0) / args.steps * 1e3
    log(f"graph replay: {graph_ms:.3f} ms/step")

    tile = list(ctx.get_tile(W, H, B, mesh.n_tris))
    res = {
        "metric": METRIC,
        "value": B * args.steps / wall,
        "unit": "pose-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "differentiation: 640x480 scan vs 1,021,734-triangle meshified room map, "
                               "64 poses per launch, cost + se(3) gradient + JtJ/Jtr + LM pose update",
                   "global_batch": B, "image": [W, H], "n_tris": mesh.n_tris, "eps": eps,
                   "tile": tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(tile),
                     "valu_issue_frac_profiled": profiled_traffic(tile, "valu_issue_frac"),
                     "kernel": "k_raster (grad)", "avg_launch_ms": avg_s * 1e3,
                     "bytes_per_launch": bytes_launch, "visible_tris_per_pose": float(t_vis.mean()),
                     "k_bin": {"avg_launch_ms": bin_s * 1e3, "bytes_per_launch": bin_bytes,
                               "achieved": bin_bytes / bin_s / 1e9, "frac": bin_bytes / bin_s / 1e9 / HBM_PEAK_GBS,
                               "traffic": profiled_traffic(tile, "bin_bytes_per_launch"),
                               "note": "algorithmic bytes: the visible mesh (12 B per vertex, 12 B of indices "
                                       "per triangle) once per pose"}},
        "graph_ms_per_step": graph_ms,
        "atomics": atomic_peaks(),
    }
    if res["atomics"]:
        a = res["atomics"]
        lanes = profiled_traffic(tile, "lds_atomic_lanes_per_launch")
        if lanes is not None and a["lds_min_u64_lane_ops_per_s"]:
            a["k_raster_lds_atomic_lane_ops_per_s"] = lanes / avg_s
            a["k_raster_lds_atomic_frac"] = lanes / avg_s / a["lds_min_u64_lane_ops_per_s"]
        n_glob = profiled_traffic(tile, "bin_global_atomics_per_launch")
        if n_glob is not None and a["global_atomic_add_per_s"]:
            rate = n_glob / (profiled_traffic(tile, "bin_launch_ms") * 1e-3)
            a["k_bin_global_atomics_per_s_profiled"] = rate
            a["k_bin_global_atomic_frac"] = rate / a["global_atomic_add_per_s"]
    if not args.no_alignment:
        res["alignment"] = alignment_comparison(rm, torch, w, mesh, scan, T0)
    if not args.no_icp:
        res["icp_odometry"] = icp_odometry(rm, torch, dev)
    if not args.no_configs:
        res["configs"] = {name: config_throughput(rm, torch, dev, name) for name in config_names if name != "uneven"}
        if "uneven" in config_names:
            res["configs"]["uneven"] = uneven_stream(rm, torch, dev)
    if not args.no_trajectory:
        res["trajectory"] = trajectory_c5(rm, torch, dev)
    if not args.no_color:
        res["color"] = color_term(rm, torch, dev, w, mesh, scan, T0)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a pixel sample")
        res["cpu_baseline"] = cpu_baseline(w, torch)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
