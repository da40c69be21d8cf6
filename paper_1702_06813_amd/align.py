"""Pose alignment drivers over the library's batched scoring.

batched_align  -- many independent alignments at once: every iteration is one
                  rm_align_cost_grad launch over all poses followed by the
                  on-device pose update (Levenberg-Marquardt or Adam), with
                  the inlier threshold eps annealed geometrically; the whole
                  iteration sequence can be captured once as a hipGraph and
                  replayed.
plain_align    -- the paper's optimizer for its own cost (Sec. IV-C): a
                  derivative-free hybrid of an initial gradient descent (finite
                  differences), Nelder-Mead iterations and coordinate descent
                  near the minimum, minimizing E(X) of Table I with one render
                  (one rm_align_cost launch for a single pose) per evaluation.
batched_plain_align -- the same optimizer for many alignments in lockstep,
                  one launch per round of evaluations over all of them.
icp_align      -- render-accelerated point-to-plane ICP (Sec. V): per
                  iteration one rm_icp_cost_grad launch over all poses
                  (render, projective association, point-to-plane blocks) and
                  the on-device Levenberg-Marquardt update.
sequential_depth_alignment -- Sec. V-B over a sequence of depth images: the
                  relative pose of every consecutive pair, all pairs solved in
                  the same launches (each pair's model placed at its own
                  offset in space so that frustum culling keeps them apart).

Pose increments x = (upsilon, omega) are applied on the right, T exp(x).
"""
from __future__ import annotations

import numpy as np
import torch

from . import rendermap as R


def eps_schedule(iters: int, eps0: float = 0.5, eps1: float = 0.1):
    """Geometric annealing of the inlier threshold from eps0 to eps1.  At
    10 cm / 5 deg most residuals exceed the paper's 0.1 m and carry no
    gradient; a wide threshold first, then the paper's value, keeps the
    basin wide and ends on the paper's cost."""
    if iters <= 1:
        return [eps1]
    return [float(eps0 * (eps1 / eps0) ** (k / (iters - 1))) for k in range(iters)]


class BatchedAligner:
    """Fixed-shape batched alignment (mesh, scans and pose count fixed), with
    optional hipGraph capture of the full iteration sequence."""

    def __init__(self, mesh, scans, n_poses, iters=20, eps=(0.5, 0.1), method="gn", lam=1e-3, lr=(0.04, 0.002),
                 poses_per_scan=None, device=None, betas=(0.5, 0.9)):
        """method "gn" (Levenberg-Marquardt, damping lam) or "adam" (step size
        lr, or (lr0, lr1) for a geometric schedule from lr0 to lr1; moment
        decays betas).  The Adam defaults are the best of a small sweep on
        the Kinect-like map from 10 cm / 5 deg in 20 iterations."""
        self.mesh, self.scans = mesh, scans
        self.dev = mesh.xyz.device if device is None else device
        self.iters, self.method, self.lam = iters, method, lam
        self.lrs = eps_schedule(iters, *lr) if isinstance(lr, (tuple, list)) else [float(lr)] * iters
        self.betas = betas
        self.eps = eps_schedule(iters, *eps)
        self.pps = poses_per_scan
        self.T = torch.empty((n_poses, 12), dtype=torch.float64, device=self.dev)
        self.out = torch.empty((n_poses, R.OUT_STRIDE), dtype=torch.float64, device=self.dev)
        self.m = torch.zeros((n_poses, 6), dtype=torch.float64, device=self.dev)
        self.v = torch.zeros((n_poses, 6), dtype=torch.float64, device=self.dev)
        self.graph = None

    def _iterations(self):
        for k, e in enumerate(self.eps):
            R.align_cost_grad(self.mesh, self.scans, self.T, e, poses_per_scan=self.pps, out=self.out)
            if self.method == "gn":
                R.gn_step(self.out, self.T, self.lam)
            else:
                R.adam_step(self.out, self.T, self.m, self.v, k + 1, self.lrs[k], *self.betas)

    def run(self, T0: torch.Tensor, use_graph=False):
        """Aligns every pose of T0 ([P,12] f64 on the device); returns T (in place buffer)."""
        self.T.copy_(T0.reshape(-1, 12))
        self.m.zero_()
        self.v.zero_()
        if not use_graph:
            self._iterations()
            return self.T
        if self.graph is None:
            self._iterations()                   # sizes scratch; then reset and capture
            torch.cuda.synchronize(self.dev)
            self.T.copy_(T0.reshape(-1, 12))
            self.m.zero_()
            self.v.zero_()
            torch.cuda.synchronize(self.dev)
            g = R.Graph(self.dev)
            with g:
                self._iterations()
            self.graph = g
            self.T.copy_(T0.reshape(-1, 12))
            self.m.zero_()
            self.v.zero_()
        self.graph.replay()
        return self.T


class TrajectoryAligner:
    """Scan-to-map alignment of a stream of scans of mixed resolutions: scans
    are taken in batches of up to MAX_SCANS per launch (one pose each), every
    batch's whole iteration sequence (cost + gradient + Gauss-Newton blocks,
    Levenberg-Marquardt update, eps schedule) replayed from one hipGraph per
    batch shape.  A batch's scan images are copied into fixed staging images
    of its shape (ordered by resolution), so that the graph of a shape serves
    every batch of that shape."""

    def __init__(self, mesh, iters=20, eps=(0.5, 0.1), lam=1e-3, batch=None):
        self.mesh = mesh
        self.iters, self.eps, self.lam = iters, eps, lam
        self.batch = batch or R.MAX_SCANS
        self.shapes = {}

    def _shape(self, cams):
        key = tuple((int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy))
                    for c in cams)
        if key not in self.shapes:
            dev = self.mesh.xyz.device
            stage = [R.Scan(torch.empty((int(c.height), int(c.width)), dtype=torch.float32, device=dev),
                            torch.empty((int(c.height), int(c.width)), dtype=torch.uint8, device=dev), c)
                     for c in cams]
            al = BatchedAligner(self.mesh, stage, len(cams), self.iters, self.eps, "gn", self.lam,
                                poses_per_scan=[1] * len(cams))
            self.shapes[key] = (stage, al)
        return self.shapes[key]

    def run(self, scans, T0, use_graph=True):
        """scans: list of R.Scan (device scan images); T0: [N,12] or [N,3,4]
        initial poses (host or device).  Returns [N,3,4] f64 host poses and
        the number of launches of the cost kernel."""
        dev = self.mesh.xyz.device
        T0 = torch.as_tensor(np.asarray(T0, np.float64).reshape(-1, 12) if not torch.is_tensor(T0) else T0,
                             device=dev).reshape(-1, 12)
        out = torch.empty_like(T0)
        launches = 0
        for b0 in range(0, len(scans), self.batch):
            idx = list(range(b0, min(b0 + self.batch, len(scans))))
            idx.sort(key=lambda j: (int(scans[j].cam.height), int(scans[j].cam.width)))
            stage, al = self._shape([scans[j].cam for j in idx])
            for st, j in zip(stage, idx):
                st.depth.copy_(scans[j].depth)
                st.cls.copy_(scans[j].cls)
            T = al.run(T0[idx], use_graph=use_graph)
            out[idx] = T
            launches += self.iters
        return out.cpu().numpy().reshape(-1, 3, 4), launches


def batched_align(mesh, scans, T0, iters=20, eps=(0.5, 0.1), method="gn", lam=1e-3, lr=(0.04, 0.002),
                  poses_per_scan=None):
    a = BatchedAligner(mesh, scans, T0.reshape(-1, 12).shape[0], iters, eps, method, lam, lr, poses_per_scan)
    return a.run(T0).clone()


# ---------------------------------------------------------------------------- derivative-free (the paper's)
#
# The optimizers are generators: each yields the next point it needs and is
# sent that point's cost, and returns (x, fx, evaluations).  One generator
# driven by a function is the plain form; many driven together share one
# batched launch per round of evaluations (batched_plain_align).

def _nelder_mead(x0, scale, max_evals, tol=1e-9):
    """Standard Nelder-Mead (reflection 1, expansion 2, contraction 1/2,
    shrink 1/2) from the simplex x0 + scale_i e_i."""
    n = len(x0)
    pts = [np.array(x0, float)] + [np.array(x0, float) + scale[i] * np.eye(n)[i] for i in range(n)]
    vals = []
    for p in pts:
        vals.append((yield p))
    evals = n + 1
    while evals < max_evals:
        order = np.argsort(vals)
        pts = [pts[i] for i in order]
        vals = [vals[i] for i in order]
        if abs(vals[-1] - vals[0]) <= tol and np.max(np.abs(np.array(pts[1:]) - pts[0])) <= tol:
            break
        c = np.mean(pts[:-1], axis=0)
        xr = c + (c - pts[-1])
        fr = yield xr
        evals += 1
        if fr < vals[0]:
            xe = c + 2.0 * (c - pts[-1])
            fe = yield xe
            evals += 1
            if fe < fr:
                pts[-1], vals[-1] = xe, fe
            else:
                pts[-1], vals[-1] = xr, fr
        elif fr < vals[-2]:
            pts[-1], vals[-1] = xr, fr
        else:
            xc = c + 0.5 * (pts[-1] - c) if fr >= vals[-1] else c + 0.5 * (xr - c)
            fc = yield xc
            evals += 1
            if fc < min(fr, vals[-1]):
                pts[-1], vals[-1] = xc, fc
            else:
                for i in range(1, len(pts)):
                    pts[i] = pts[0] + 0.5 * (pts[i] - pts[0])
                    vals[i] = yield pts[i]
                    evals += 1
    i = int(np.argmin(vals))
    return pts[i], vals[i], evals


def _coordinate_descent(x0, f0, step, max_evals, shrink=0.5, min_step=1e-4):
    """Coordinate descent with per-axis step halving near the minimum."""
    x, fx, evals = np.array(x0, float), f0, 0
    step = np.array(step, float)
    while evals < max_evals and np.any(step > min_step):
        for i in range(len(x)):
            if step[i] <= min_step:
                continue
            for sgn in (+1.0, -1.0):
                y = x.copy(); y[i] += sgn * step[i]
                fy = yield y
                evals += 1
                if fy < fx:
                    x, fx = y, fy
                    break
            else:
                step[i] *= shrink
            if evals >= max_evals:
                break
    return x, fx, evals


def _hybrid(n=6, budget=700, fd_step=(0.02, 0.02, 0.02, 0.02, 0.02, 0.02),
            simplex=(0.05, 0.05, 0.05, 0.05, 0.05, 0.05), gd_iters=2, nm_share=0.6):
    """Initial gradient descent by central differences with a backtracking
    line search, then Nelder-Mead, then coordinate descent (Sec. IV-C)."""
    x = np.zeros(n)
    fx = yield x
    evals = 1
    h = np.asarray(fd_step, float)
    for _ in range(gd_iters):
        g = np.zeros(n)
        for i in range(n):
            e = np.zeros(n); e[i] = h[i]
            fp = yield x + e
            fm = yield x - e
            g[i] = (fp - fm) / (2 * h[i])
            evals += 2
        gn = np.linalg.norm(g / h)
        if gn == 0:
            break
        d = -(g / h) / gn * h * 4.0           # a few finite-difference steps along -grad
        t = 1.0
        for _ in range(6):
            y = x + t * d
            fy = yield y
            evals += 1
            if fy < fx:
                x, fx = y, fy
                break
            t *= 0.5
    x, fx, e1 = yield from _nelder_mead(x, np.asarray(simplex, float), int((budget - evals) * nm_share) + evals)
    evals += e1
    x2, fx2, e2 = yield from _coordinate_descent(x, fx, np.asarray(simplex, float) * 0.25, budget - evals)
    return (x2, fx2, evals + e2) if fx2 <= fx else (x, fx, evals + e2)


# ---------------------------------------------------------------------------- speculative batches
#
# The same optimizer asking, at each step, for every point the next decision
# may need: each yield is a list of points and is sent the list of their
# costs (one batched launch).  Decisions are then taken in the sequential
# order from those costs, so the trajectory, the result and the counted
# evaluations are exactly those of the one-point generators above; points
# the sequential form would not have evaluated are discarded uncounted.
#   initial gradient descent: x with its 2n-point central-difference stencil,
#     then the six backtracking steps of the line search, then the next stencil;
#   Nelder-Mead: the initial simplex, then per iteration the reflection, the
#     expansion and both contractions (and the n shrink points only if needed);
#   coordinate descent: the +/- probes of every remaining axis of the sweep at
#     the current point, up to the first accepted probe.

def _stencil(x, h):
    pts = []
    for i in range(len(x)):
        e = np.zeros(len(x)); e[i] = h[i]
        pts += [x + e, x - e]
    return pts


def _nelder_mead_b(x0, scale, max_evals, tol=1e-9):
    n = len(x0)
    pts = [np.array(x0, float)] + [np.array(x0, float) + scale[i] * np.eye(n)[i] for i in range(n)]
    vals = list((yield list(pts)))
    evals = n + 1
    while evals < max_evals:
        order = np.argsort(vals)
        pts = [pts[i] for i in order]
        vals = [vals[i] for i in order]
        if abs(vals[-1] - vals[0]) <= tol and np.max(np.abs(np.array(pts[1:]) - pts[0])) <= tol:
            break
        c = np.mean(pts[:-1], axis=0)
        xr = c + (c - pts[-1])
        xe = c + 2.0 * (c - pts[-1])
        xc_out = c + 0.5 * (xr - c)
        xc_in = c + 0.5 * (pts[-1] - c)
        fr, fe, fco, fci = (yield [xr, xe, xc_out, xc_in])
        evals += 1
        if fr < vals[0]:
            evals += 1
            if fe < fr:
                pts[-1], vals[-1] = xe, fe
            else:
                pts[-1], vals[-1] = xr, fr
        elif fr < vals[-2]:
            pts[-1], vals[-1] = xr, fr
        else:
            xc, fc = (xc_in, fci) if fr >= vals[-1] else (xc_out, fco)
            evals += 1
            if fc < min(fr, vals[-1]):
                pts[-1], vals[-1] = xc, fc
            else:
                shr = [pts[0] + 0.5 * (pts[i] - pts[0]) for i in range(1, len(pts))]
                vs = yield shr
                for i in range(1, len(pts)):
                    pts[i], vals[i] = shr[i - 1], vs[i - 1]
                    evals += 1
    i = int(np.argmin(vals))
    return pts[i], vals[i], evals


def _coordinate_descent_b(x0, f0, step, max_evals, shrink=0.5, min_step=1e-4):
    x, fx, evals = np.array(x0, float), f0, 0
    step = np.array(step, float)
    n = len(x)
    while evals < max_evals and np.any(step > min_step):
        i = 0
        while i < n:
            axes = [k for k in range(i, n) if step[k] > min_step]
            if not axes:
                break
            probes = []
            for k in axes:
                for sgn in (+1.0, -1.0):
                    y = x.copy(); y[k] += sgn * step[k]
                    probes.append(y)
            v = yield probes
            i = n                                  # the sweep ends unless a probe is accepted
            for j, k in enumerate(axes):
                accepted = False
                for s in range(2):
                    evals += 1
                    if v[2 * j + s] < fx:
                        x, fx = probes[2 * j + s], v[2 * j + s]
                        accepted = True
                        break
                if not accepted:
                    step[k] *= shrink
                if evals >= max_evals:
                    break
                if accepted:
                    i = k + 1                      # later axes from the new point
                    break
            if evals >= max_evals:
                break
    return x, fx, evals


def _hybrid_b(n=6, budget=700, fd_step=(0.02, 0.02, 0.02, 0.02, 0.02, 0.02),
              simplex=(0.05, 0.05, 0.05, 0.05, 0.05, 0.05), gd_iters=2, nm_share=0.6):
    """_hybrid asking for points in speculative batches (same result)."""
    x = np.zeros(n)
    h = np.asarray(fd_step, float)
    first = yield [x] + _stencil(x, h)
    fx = first[0]
    evals = 1
    for it in range(gd_iters):
        v = first[1:] if it == 0 else (yield _stencil(x, h))
        g = np.zeros(n)
        for i in range(n):
            g[i] = (v[2 * i] - v[2 * i + 1]) / (2 * h[i])
            evals += 2
        gn = np.linalg.norm(g / h)
        if gn == 0:
            break
        d = -(g / h) / gn * h * 4.0
        ys, t = [], 1.0
        for _ in range(6):
            ys.append(x + t * d)
            t *= 0.5
        vy = yield ys
        for y, fy in zip(ys, vy):
            evals += 1
            if fy < fx:
                x, fx = y, fy
                break
    x, fx, e1 = yield from _nelder_mead_b(x, np.asarray(simplex, float), int((budget - evals) * nm_share) + evals)
    evals += e1
    x2, fx2, e2 = yield from _coordinate_descent_b(x, fx, np.asarray(simplex, float) * 0.25, budget - evals)
    return (x2, fx2, evals + e2) if fx2 <= fx else (x, fx, evals + e2)


def _drive_b(gen, f):
    """Drives a batch generator with f(list of points) -> list of costs;
    returns (result, batches)."""
    batches = 0
    try:
        pts = next(gen)
        while True:
            batches += 1
            pts = gen.send([float(v) for v in f(pts)])
    except StopIteration as stop:
        return stop.value, batches


def hybrid_minimize_batched(f_batch, n=6, budget=700, **kw):
    """The hybrid optimizer with speculative batches: f_batch(list of points)
    returns their costs.  Returns (x, fx, evals, batches), (x, fx, evals)
    equal to hybrid_minimize's."""
    (x, fx, ev), nb = _drive_b(_hybrid_b(n, budget, **kw), f_batch)
    return x, fx, ev, nb


def lockstep_batches(gens, evaluate):
    """lockstep for batch generators: each round, evaluate(ks, lists of
    points) receives the unfinished instances and their batches and returns
    one list of costs per instance.  Returns (results, rounds)."""
    pending = [next(g) for g in gens]
    result = [None] * len(gens)
    rounds = 0
    while True:
        act = [k for k in range(len(gens)) if result[k] is None]
        if not act:
            return result, rounds
        vals = evaluate(act, [pending[k] for k in act])
        rounds += 1
        for k, v in zip(act, vals):
            try:
                pending[k] = gens[k].send([float(x) for x in v])
            except StopIteration as stop:
                result[k] = stop.value


def _drive(gen, f):
    try:
        x = next(gen)
        while True:
            x = gen.send(f(x))
    except StopIteration as stop:
        return stop.value


def nelder_mead(f, x0, scale, max_evals, tol=1e-9):
    """Nelder-Mead on f; returns (x, fx, evals)."""
    return _drive(_nelder_mead(x0, scale, max_evals, tol), f)


def coordinate_descent(f, x0, f0, step, max_evals, shrink=0.5, min_step=1e-4):
    """Coordinate descent on f from (x0, f0); returns (x, fx, evals)."""
    return _drive(_coordinate_descent(x0, f0, step, max_evals, shrink, min_step), f)


def hybrid_minimize(f, n=6, budget=700, **kw):
    """The paper's hybrid optimizer on f from x = 0; returns (x, fx, evals)."""
    return _drive(_hybrid(n, budget, **kw), f)


def plain_align_batched(mesh, scan, T0, eps=0.1, budget=700, weights=None, color_tol=0.0):
    """The paper's optimizer for one alignment with its independent points
    evaluated together: every batch of the speculative hybrid optimizer (the
    finite-difference stencil, the line-search steps, the initial simplex,
    the Nelder-Mead candidates, the coordinate-descent probes) is one
    rm_align_cost launch.  Same trajectory, pose, cost and evaluation count
    as plain_align.  Returns (T [3,4] numpy, E, evaluations, launches)."""
    dev = mesh.xyz.device
    T0d = torch.as_tensor(np.asarray(T0, np.float64).reshape(1, 12), device=dev)

    def f(xs):
        X = torch.from_numpy(np.stack(xs)).to(dev)
        Td = R.se3_retract(T0d.expand(len(xs), 12).contiguous(), X)
        out = R.align_cost(mesh, scan, Td, eps, color_tol=color_tol)
        v = out[:, R.OUT_E_TABLE] if weights is None else R.table_cost_weighted(out, weights)
        return v.cpu().numpy()

    x, fx, evals, launches = hybrid_minimize_batched(f, budget=budget)
    xd = torch.from_numpy(np.asarray(x, np.float64).reshape(1, 6)).to(dev)
    return R.se3_retract(T0d, xd).cpu().numpy().reshape(3, 4), fx, evals, launches


def plain_align(mesh, scan, T0, eps=0.1, budget=700, weights=None, color_tol=0.0):
    """The paper's plain form: minimize E(X) (Table I) of one pose with the
    derivative-free hybrid optimizer, one single-pose render per evaluation.
    weights: optional nine Table I cell weights, or eleven with the color
    reward and penalty weights (rm_table_cost_weighted; Sec. IV-C suggests
    reweighting the penalties and rewards, and color costs and rewards),
    None for E(X); color_tol: the color term's agreement threshold.
    T0: [12] or [3,4] (host).  Returns (T [3,4] numpy, E, evaluations)."""
    dev = mesh.xyz.device
    T0d = torch.as_tensor(np.asarray(T0, np.float64).reshape(1, 12), device=dev)
    xd = torch.zeros((1, 6), dtype=torch.float64, device=dev)
    Td = torch.empty_like(T0d)
    out = torch.empty((1, R.OUT_STRIDE), dtype=torch.float64, device=dev)

    def f(x):
        xd.copy_(torch.from_numpy(np.asarray(x, np.float64).reshape(1, 6)))
        R.se3_retract(T0d, xd, out=Td)
        R.align_cost(mesh, scan, Td, eps, out=out, color_tol=color_tol)
        if weights is not None:
            return float(R.table_cost_weighted(out, weights)[0].item())
        return float(out[0, R.OUT_E_TABLE].item())

    x, fx, evals = hybrid_minimize(f, budget=budget)
    xd.copy_(torch.from_numpy(np.asarray(x, np.float64).reshape(1, 6)))
    R.se3_retract(T0d, xd, out=Td)
    return Td.cpu().numpy().reshape(3, 4), fx, evals


def lockstep(gens, evaluate):
    """Drives optimizer generators together: each round, evaluate(ks, xs)
    receives the unfinished instances and their next points and returns their
    costs.  Returns (results per instance, rounds)."""
    pending = [next(g) for g in gens]
    result = [None] * len(gens)
    rounds = 0
    while True:
        act = [k for k in range(len(gens)) if result[k] is None]
        if not act:
            return result, rounds
        vals = evaluate(act, [pending[k] for k in act])
        rounds += 1
        for k, v in zip(act, vals):
            try:
                pending[k] = gens[k].send(float(v))
            except StopIteration as stop:
                result[k] = stop.value


def batched_plain_align(mesh, scans, T0, eps=0.1, budget=700, scan_of=None, weights=None, speculative=False,
                        color_tol=0.0):
    """The paper's optimizer for many alignments at once: every instance runs
    the same hybrid optimizer as plain_align, and each round evaluates the
    next point of every unfinished instance in one launch (T0: [K,3,4] or
    [K,12] host poses; scans: one scan, or a list with scan_of[k] the scan of
    instance k).  Each instance evaluates exactly the points plain_align
    would.  With speculative=True every instance contributes its whole
    speculative batch (plain_align_batched) to each round's launch: fewer
    launches, same results.  Returns (T [K,3,4] numpy, E [K], evaluations
    [K], launches)."""
    dev = mesh.xyz.device
    T0 = np.asarray(T0, np.float64).reshape(-1, 12)
    K = T0.shape[0]
    if isinstance(scans, R.Scan):
        scans, scan_of = [scans], [0] * K
    scan_of = np.asarray(scan_of if scan_of is not None else [0] * K)
    T0d = torch.from_numpy(T0).to(dev)

    def evaluate(ks, xs):
        # the active instances grouped by scan, in scan order, as one batched launch
        order = sorted(range(len(ks)), key=lambda j: scan_of[ks[j]])
        kk = [ks[j] for j in order]
        used = sorted(set(scan_of[kk].tolist()))
        counts = [int((scan_of[kk] == sc).sum()) for sc in used]
        X = torch.from_numpy(np.stack([xs[j] for j in order])).to(dev)
        Td = R.se3_retract(T0d[kk].contiguous(), X)
        out = R.align_cost(mesh, [scans[sc] for sc in used], Td, eps, poses_per_scan=counts, color_tol=color_tol)
        v = (out[:, R.OUT_E_TABLE] if weights is None else R.table_cost_weighted(out, weights)).cpu().numpy()
        res = np.empty(len(ks))
        res[order] = v
        return res

    if speculative:
        def evaluate_b(ks, batches):
            # every point of every active instance's batch in one launch
            flat_k = [k for k, b in zip(ks, batches) for _ in b]
            flat_x = [x for b in batches for x in b]
            v = evaluate(flat_k, flat_x)
            out, o = [], 0
            for b in batches:
                out.append(v[o:o + len(b)]); o += len(b)
            return out
        result, launches = lockstep_batches([_hybrid_b(budget=budget) for _ in range(K)], evaluate_b)
    else:
        result, launches = lockstep([_hybrid(budget=budget) for _ in range(K)], evaluate)
    X = torch.from_numpy(np.stack([r[0] for r in result])).to(dev)
    T = R.se3_retract(T0d, X).cpu().numpy().reshape(K, 3, 4)
    return T, np.array([r[1] for r in result]), np.array([r[2] for r in result]), launches


def pose_errors(T, T_true):
    """Translation error (m) and rotation angle error (rad) of each pose."""
    T = np.asarray(T, np.float64).reshape(-1, 3, 4)
    Tt = np.asarray(T_true, np.float64).reshape(3, 4)
    dt = np.linalg.norm(T[:, :, 3] - Tt[:, 3], axis=1)
    Rrel = np.einsum("kji,jl->kil", T[:, :, :3], Tt[:, :3])
    ang = np.arccos(np.clip((np.trace(Rrel, axis1=1, axis2=2) - 1) / 2, -1, 1))
    return dt, ang


# ---------------------------------------------------------------------------- render-accelerated ICP (Sec. V)

def icp_align(mesh, vnormals, scans, T0, tol=0.1, iters=10, lam=1e-6, poses_per_scan=None):
    """Point-to-plane ICP with projective association for every pose at once.
    Returns (T [P,3,4] f64 device, last result records [P,48])."""
    T = R._poses(T0, mesh.xyz.device).clone()
    out = torch.empty((T.shape[0], R.OUT_STRIDE), dtype=torch.float64, device=T.device)
    for _ in range(iters):
        R.icp_cost_grad(mesh, scans, T, vnormals, tol, poses_per_scan, out)
        R.gn_step(out, T, lam)
    return T.view(-1, 3, 4), out


def _pair_offset(k, spacing):
    """Translation placing pair k's model at its own spot of a 4 x 4 x n grid."""
    return np.array([(k % 4) * spacing, ((k // 4) % 4) * spacing, (k // 16) * spacing], np.float64)


def prepare_pairs(depths, cam, ks, factor=2, z_min=0.1, z_max=8.0, stride=1, max_edge=0.1, sigma=1.0, radius=2,
                  spacing=50.0, ds=None):
    """Steps 1-2 of Sec. V-B for the consecutive pairs (k, k+1), k in ``ks``
    (at most MAX_SCANS): the model of each pair is the mesh of downsampled
    image k, placed at its own offset and carrying its Eq. (2) normals; the
    scan is downsampled image k+1.  Returns (mesh, vertex normals, scans,
    offset poses [n,3,4], downsampled camera)."""
    cam2 = R.downsample_camera(cam, factor)
    if ds is None:
        ds = {}
    for k in ks:
        for j in (k, k + 1):
            if j not in ds:
                ds[j] = R.depth_downsample(depths[j], factor, z_max)
    meshes, vns, offs = [], [], []
    for i, k in enumerate(ks):
        To = np.zeros((3, 4))
        To[:, :3] = np.eye(3)
        To[:, 3] = _pair_offset(i, spacing)
        offs.append(To)
        meshes.append(R.mesh_from_range(ds[k], cam2, To, stride, z_min, z_max, max_edge, 0))
        vns.append(R.vertex_normals(R.depth_normals(ds[k], cam2, sigma, radius), stride, To))
    mesh = R.Mesh.concat(meshes).prepare()
    vn = torch.cat(vns).contiguous()
    scans = [R.scan_image(ds[k + 1], z_min, z_max, cam=cam2) for k in ks]
    return mesh, vn, scans, np.stack(offs), cam2


def sequential_depth_alignment(depths, cam, factor=2, z_min=0.1, z_max=8.0, stride=1, max_edge=0.1,
                               sigma=1.0, radius=2, tol=0.1, iters=10, lam=1e-6, spacing=50.0, init=None):
    """Relative poses between consecutive depth images (Sec. V-B).

    depths: list of device [H, W] f32 depth images of camera ``cam``.
    For each pair (i, i+1): downsample both by ``factor`` dropping points
    beyond z_max (step 1), normals of image i by Eq. (2) (step 2), its mesh
    carrying those normals rendered from the current estimate of image i+1's
    pose (step 3), point-to-plane ICP of image i+1's points (step 4),
    repeated ``iters`` times (step 5).  ``init``: optional [N-1, 3, 4] initial
    relative poses (identity otherwise).  Returns ([N-1, 3, 4] numpy relative
    poses T_{i,i+1} (frame i+1 in frame i), last result records)."""
    dev = depths[0].device
    n_pairs = len(depths) - 1
    T_all, outs, ds = [], [], {}
    for b0 in range(0, n_pairs, R.MAX_SCANS):
        ks = list(range(b0, min(b0 + R.MAX_SCANS, n_pairs)))
        mesh, vn, scans, offs, _ = prepare_pairs(depths, cam, ks, factor, z_min, z_max, stride, max_edge, sigma,
                                                 radius, spacing, ds)
        T0 = offs.copy()
        if init is not None:
            T0 = np.stack([np.vstack([o, [0, 0, 0, 1]]) @ np.vstack([np.asarray(init[k]), [0, 0, 0, 1]])
                           for o, k in zip(offs, ks)])[:, :3]
        T, out = icp_align(mesh, vn, scans, torch.from_numpy(np.ascontiguousarray(T0.reshape(-1, 12))).to(dev),
                           tol, iters, lam, [1] * len(ks))
        Tn = T.cpu().numpy()
        for j in range(len(ks)):
            Trel = Tn[j].copy()
            Trel[:, 3] -= offs[j][:, 3]
            T_all.append(Trel)
        outs.append(out)
    return np.stack(T_all), torch.cat(outs)
