"""ctypes binding of librendermap.so (the C ABI in include/rendermap.h).

Argument marshalling only: tensors are checked (device, dtype, layout) and
their device pointers handed to the library together with PyTorch's current
HIP stream; every step of the pose-scoring path runs in the library's HIP
kernels.  There is no CPU fallback: if the library is missing or no GPU is
present, every call raises.
"""
from __future__ import annotations

import ctypes
import threading
from dataclasses import dataclass
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "librendermap.so"

RM_OK, RM_ERR_INVALID_ARG, RM_ERR_OOM, RM_ERR_DEVICE, RM_ERR_CAPACITY, RM_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FO, FU, UO, NONE = 0, 1, 2, 3
OUT_E_TABLE, OUT_E_SOFT, OUT_COUNTS, OUT_N_ACTIVE = 0, 1, 2, 11
OUT_GRAD, OUT_JTR, OUT_JTJ, OUT_N_VISIBLE, OUT_STRIDE = 12, 18, 24, 45, 48
OUT_COLOR_REWARD, OUT_COLOR_PENALTY = 46, 47
OUT_ICP_COST, OUT_ICP_SSE, OUT_ICP_N_SCAN, OUT_ICP_N_MODEL = 0, 1, 2, 3
MAX_NORMAL_RADIUS = 8
MAX_SCANS = 32
CLUSTER_TRIS = 256

ABI_SYMBOLS = [
    "rm_ctx_create", "rm_ctx_destroy", "rm_ctx_set_stream", "rm_last_error", "rm_set_tile", "rm_autotune",
    "rm_get_tile", "rm_set_schedule", "rm_profile", "rm_profile_read", "rm_graph_begin", "rm_graph_end", "rm_graph_launch", "rm_graph_destroy", "rm_scan_image",
    "rm_mesh_from_range", "rm_mesh_clusters_size", "rm_mesh_clusters", "rm_render_depth", "rm_align_cost",
    "rm_align_cost_grad", "rm_gn_step", "rm_adam_step", "rm_se3_retract", "rm_depth_downsample",
    "rm_depth_normals", "rm_vertex_normals", "rm_icp_cost_grad", "rm_table_cost_weighted", "rm_set_bin_cap",
    "rm_set_bin_pool",
    "rm_align_cost_grad_noalloc", "rm_profile_read_binning",
]
TABLE_WEIGHTS = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0, 0.0, 0.0, 0.0)   # Table I as printed: reproduces E_TABLE
N_WEIGHTS = 11            # nine Table I cells, then the color reward and penalty


class RenderMapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rendermap error {code}: {msg}")
        self.code = code


class CCamera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("z_near", ctypes.c_float),
                ("z_far", ctypes.c_float)]


class CMesh(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("n_vertices", ctypes.c_int64), ("tri", ctypes.c_void_p),
                ("cls", ctypes.c_void_p), ("n_tris", ctypes.c_int64), ("clusters", ctypes.c_void_p),
                ("color", ctypes.c_void_p)]


class CScan(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("cls", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("cam", CCamera),
                ("color", ctypes.c_void_p)]


class CCostParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("flags", ctypes.c_int32), ("color_tol", ctypes.c_float)]


_lib = None
_lib_lock = threading.Lock()


def load_library(path: Path | str | None = None):
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is not None:
            return _lib
        p = Path(path) if path else LIB_PATH
        if not p.exists():
            raise RuntimeError(f"{p} not found: build it first (python -m paper_1702_06813_amd.build)")
        L = ctypes.CDLL(str(p))
        V, I32, I64, D, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
        sig = {
            "rm_ctx_create": [I32, ctypes.POINTER(V)],
            "rm_ctx_destroy": [V],
            "rm_ctx_set_stream": [V, V],
            "rm_set_tile": [V, I32, I32],
            "rm_autotune": [V, I32],
            "rm_set_schedule": [V, I32],
            "rm_set_bin_cap": [V, I32],
            "rm_set_bin_pool": [V, I64],
            "rm_get_tile": [V, I32, I32, I32, I64, ctypes.POINTER(I32), ctypes.POINTER(I32)],
            "rm_profile": [V, I32],
            "rm_profile_read": [V, ctypes.POINTER(I64), ctypes.POINTER(D)],
            "rm_profile_read_binning": [V, ctypes.POINTER(I64), ctypes.POINTER(D)],
            "rm_graph_begin": [V],
            "rm_graph_end": [V, ctypes.POINTER(V)],
            "rm_graph_launch": [V, V],
            "rm_graph_destroy": [V],
            "rm_scan_image": [V, V, I32, I32, F, F, V, V],
            "rm_mesh_from_range": [V, V, CCamera, V, I32, I32, F, F, F, V, V, V, I64, ctypes.POINTER(I64),
                                   ctypes.POINTER(I64)],
            "rm_mesh_clusters": [V, ctypes.POINTER(CMesh), V],
            "rm_render_depth": [V, ctypes.POINTER(CMesh), CCamera, V, I32, V, V, V],
            "rm_align_cost": [V, ctypes.POINTER(CMesh), ctypes.POINTER(CScan), I32, V, V, CCostParams, V],
            "rm_align_cost_grad": [V, ctypes.POINTER(CMesh), ctypes.POINTER(CScan), I32, V, V, CCostParams, V],
            "rm_align_cost_grad_noalloc": [V, ctypes.POINTER(CMesh), ctypes.POINTER(CScan), I32, V, V, CCostParams,
                                           V],
            "rm_gn_step": [V, V, I32, D, V, V],
            "rm_adam_step": [V, V, I32, D, D, D, I32, V, V, V],
            "rm_se3_retract": [V, V, V, I32, V],
            "rm_depth_downsample": [V, V, I32, I32, I32, F, V],
            "rm_depth_normals": [V, V, I32, I32, F, F, F, I32, V],
            "rm_vertex_normals": [V, V, I32, I32, I32, V, V],
            "rm_icp_cost_grad": [V, ctypes.POINTER(CMesh), V, ctypes.POINTER(CScan), I32, V, V, F, V],
            "rm_table_cost_weighted": [V, V, I32, V, V],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.rm_last_error.argtypes = [V]
        L.rm_last_error.restype = ctypes.c_char_p
        L.rm_mesh_clusters_size.argtypes = [I64]
        L.rm_mesh_clusters_size.restype = I64
        _lib = L
        return L


def _check(rc, ctx_handle=None):
    if rc != RM_OK:
        msg = load_library().rm_last_error(ctx_handle)
        raise RenderMapError(rc, msg.decode() if msg else "")


class Context:
    """An rm_ctx bound to one GPU; calls run on PyTorch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("rendermap needs a ROCm GPU; none is available")
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        _check(self.lib.rm_ctx_create(device, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        try:
            if getattr(self, "handle", None) and self.handle.value:
                self.lib.rm_ctx_destroy(self.handle)
        except Exception:
            pass

    def call(self, name, *args):
        self.lib.rm_ctx_set_stream(self.handle, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        _check(getattr(self.lib, name)(self.handle, *args), self.handle)

    def set_tile(self, w: int, h: int):
        _check(self.lib.rm_set_tile(self.handle, w, h), self.handle)

    def set_schedule(self, mode: int):
        """rm_set_schedule: 0 automatic (persistent), 1 one workgroup per item, 2 persistent longest-first."""
        self.call("rm_set_schedule", int(mode))

    def set_bin_cap(self, cap: int):
        """rm_set_bin_cap: fixed tile-bin capacity in entries (0: adaptive)."""
        _check(self.lib.rm_set_bin_cap(self.handle, int(cap)), self.handle)

    def set_bin_pool(self, entries: int):
        """rm_set_bin_pool: overflow pool of the tile bins (-1 adaptive, 0 none,
        > 0 fixed entries)."""
        _check(self.lib.rm_set_bin_pool(self.handle, int(entries)), self.handle)

    def autotune(self, enable: bool = True):
        _check(self.lib.rm_autotune(self.handle, int(enable)), self.handle)

    def profile(self, enable: bool = True):
        """Times every rasterizer launch with HIP events on the launch stream."""
        _check(self.lib.rm_profile(self.handle, int(enable)), self.handle)

    def profile_read(self):
        """(number of timed rasterizer launches, summed milliseconds); clears."""
        self.lib.rm_ctx_set_stream(self.handle, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(self.lib.rm_profile_read(self.handle, ctypes.byref(n), ctypes.byref(ms)), self.handle)
        return n.value, ms.value

    def profile_read_binning(self):
        """(number of timed binning launches, summed milliseconds); clears."""
        self.lib.rm_ctx_set_stream(self.handle, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(self.lib.rm_profile_read_binning(self.handle, ctypes.byref(n), ctypes.byref(ms)), self.handle)
        return n.value, ms.value

    def get_tile(self, width, height, n_poses, n_tris):
        w, h = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.rm_get_tile(self.handle, width, height, n_poses, n_tris, ctypes.byref(w), ctypes.byref(h)),
               self.handle)
        return w.value, h.value


_ctxs: dict[int, Context] = {}


def context(device: int | str | torch.device | None = None) -> Context:
    if isinstance(device, str):
        device = torch.device(device)
    if device is None:
        idx = torch.cuda.current_device()
    elif isinstance(device, torch.device):
        idx = device.index if device.index is not None else torch.cuda.current_device()
    else:
        idx = int(device)
    if idx not in _ctxs:
        _ctxs[idx] = Context(idx)
    return _ctxs[idx]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must live on {device or 'a GPU'}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def ccamera(cam) -> CCamera:
    if isinstance(cam, CCamera):
        return cam
    return CCamera(cam.fx, cam.fy, cam.cx, cam.cy, int(cam.width), int(cam.height), cam.z_near, cam.z_far)


# ---------------------------------------------------------------------------- data holders

@dataclass
class Mesh:
    """Device-resident interface mesh plus its cluster bounds."""
    xyz: torch.Tensor          # [V,3] f32
    tri: torch.Tensor          # [T,3] i32
    cls: torch.Tensor          # [T] u8
    clusters: torch.Tensor | None = None
    color: torch.Tensor | None = None     # [T] f32 triangle intensities (color term)

    @property
    def n_tris(self):
        return int(self.tri.shape[0])

    def struct(self) -> CMesh:
        dev = self.xyz.device
        _need(self.xyz, torch.float32, "xyz", dev)
        _need(self.tri, torch.int32, "tri", dev)
        _need(self.cls, torch.uint8, "cls", dev)
        if self.xyz.dim() != 2 or self.xyz.shape[1] != 3 or self.tri.dim() != 2 or self.tri.shape[1] != 3:
            raise ValueError("xyz must be [V,3] and tri [T,3]")
        if self.cls.shape[0] != self.tri.shape[0]:
            raise ValueError("cls must have one entry per triangle")
        if self.color is not None:
            _need(self.color, torch.float32, "color", dev)
            if tuple(self.color.shape) != (self.tri.shape[0],):
                raise ValueError("color must have one entry per triangle")
        return CMesh(self.xyz.data_ptr(), self.xyz.shape[0], self.tri.data_ptr(), self.cls.data_ptr(),
                     self.tri.shape[0], self.clusters.data_ptr() if self.clusters is not None else None,
                     self.color.data_ptr() if self.color is not None else None)

    def prepare(self):
        """Computes the cluster bounds once (rm_mesh_clusters)."""
        ctx = context(self.xyz.device)
        n = int(load_library().rm_mesh_clusters_size(self.n_tris))
        self.clusters = torch.empty(max(n, 1), dtype=torch.uint8, device=self.xyz.device)
        m = CMesh(self.xyz.data_ptr(), self.xyz.shape[0], self.tri.data_ptr(), self.cls.data_ptr(),
                  self.tri.shape[0], None, None)
        ctx.call("rm_mesh_clusters", ctypes.byref(m), _ptr(self.clusters))
        return self

    @staticmethod
    def from_arrays(xyz, tri, cls, device="cuda"):
        return Mesh(torch.as_tensor(xyz, dtype=torch.float32).contiguous().to(device),
                    torch.as_tensor(tri, dtype=torch.int32).contiguous().to(device),
                    torch.as_tensor(cls, dtype=torch.uint8).contiguous().to(device))

    @staticmethod
    def concat(meshes):
        """Union of meshes (vertex index offsets applied on the device)."""
        xyz, tri, cls, off = [], [], [], 0
        for m in meshes:
            xyz.append(m.xyz); tri.append(m.tri + off); cls.append(m.cls); off += m.xyz.shape[0]
        color = None
        if all(m.color is not None for m in meshes):
            color = torch.cat([m.color for m in meshes]).contiguous()
        return Mesh(torch.cat(xyz).contiguous(), torch.cat(tri).contiguous(), torch.cat(cls).contiguous(),
                    color=color)


@dataclass
class Scan:
    """Scan image Z_s on the device: depth d_s [H,W] f32, class c_s [H,W] u8."""
    depth: torch.Tensor
    cls: torch.Tensor
    cam: object
    mask: torch.Tensor | None = None
    color: torch.Tensor | None = None     # [H,W] f32 pixel intensities (color term), NaN = none

    def struct(self) -> CScan:
        dev = self.depth.device
        H, W = int(self.cam.height), int(self.cam.width)
        _need(self.depth, torch.float32, "scan depth", dev)
        _need(self.cls, torch.uint8, "scan cls", dev)
        if tuple(self.depth.shape) != (H, W) or tuple(self.cls.shape) != (H, W):
            raise ValueError(f"scan images must be [{H},{W}]")
        if self.mask is not None:
            _need(self.mask, torch.uint8, "mask", dev)
            if tuple(self.mask.shape) != (H, W):
                raise ValueError("mask must match the image")
        if self.color is not None:
            _need(self.color, torch.float32, "scan color", dev)
            if tuple(self.color.shape) != (H, W):
                raise ValueError("color must match the image")
        return CScan(self.depth.data_ptr(), self.cls.data_ptr(),
                     self.mask.data_ptr() if self.mask is not None else None, ccamera(self.cam),
                     self.color.data_ptr() if self.color is not None else None)


# ---------------------------------------------------------------------------- entry points

def scan_image(depth: torch.Tensor, z_min=0.5, z_max=8.0, cam=None) -> Scan:
    """rm_scan_image: the scan image (d_s, c_s) of a range image."""
    _need(depth, torch.float32, "depth", None)
    H, W = depth.shape
    ctx = context(depth.device)
    d = torch.empty_like(depth)
    c = torch.empty((H, W), dtype=torch.uint8, device=depth.device)
    ctx.call("rm_scan_image", _ptr(depth), H, W, z_min, z_max, _ptr(d), _ptr(c))
    return Scan(d, c, cam)


def _pose_host(T):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(T, dtype=np.float64).reshape(12))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def mesh_from_range(depth: torch.Tensor, cam, T_wc, stride: int, z_min=0.5, z_max=8.0, max_edge=0.1,
                    smooth_radius: int = 0) -> Mesh:
    """rm_mesh_from_range: interface mesh of one range image (synchronizes).
    smooth_radius R > 0 averages each node's depth over the (2R+1)^2 window
    pixels within 3% of it before the surfaces are built."""
    _need(depth, torch.float32, "depth", None)
    H, W = depth.shape
    if (H, W) != (int(cam.height), int(cam.width)):
        raise ValueError("depth must match the camera")
    gh, gw = -(-H // stride), -(-W // stride)
    cap = 2 * max(gh - 1, 0) * max(gw - 1, 0)
    dev = depth.device
    xyz = torch.empty((gh * gw, 3), dtype=torch.float32, device=dev)
    tri = torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev)
    cls = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    nv, nt = ctypes.c_int64(), ctypes.c_int64()
    keep, pp = _pose_host(T_wc)
    context(dev).call("rm_mesh_from_range", _ptr(depth), ccamera(cam), pp, stride, smooth_radius, z_min, z_max,
                      max_edge, _ptr(xyz), _ptr(tri), _ptr(cls), cap, ctypes.byref(nv), ctypes.byref(nt))
    n = nt.value
    return Mesh(xyz, tri[:n], cls[:n])


def _poses(T_wc, device):
    T = T_wc.reshape(-1, 12) if T_wc.dim() != 2 or T_wc.shape[1] != 12 else T_wc
    return _need(T.contiguous(), torch.float64, "T_wc", device)


def render_depth(mesh: Mesh, cam, T_wc: torch.Tensor, want=("depth", "tri", "cls")):
    """rm_render_depth: z-buffer of B poses -> dict of [B,H,W] depth/tri/cls."""
    dev = mesh.xyz.device
    T = _poses(T_wc, dev)
    B, H, W = T.shape[0], int(cam.height), int(cam.width)
    out = {}
    if "depth" in want: out["depth"] = torch.empty((B, H, W), dtype=torch.float32, device=dev)
    if "tri" in want: out["tri"] = torch.empty((B, H, W), dtype=torch.int32, device=dev)
    if "cls" in want: out["cls"] = torch.empty((B, H, W), dtype=torch.uint8, device=dev)
    m = mesh.struct()
    context(dev).call("rm_render_depth", ctypes.byref(m), ccamera(cam), _ptr(T), B, _ptr(out.get("depth")),
                      _ptr(out.get("tri")), _ptr(out.get("cls")))
    return out


def _scan_args(scans, poses_per_scan):
    scans = list(scans)
    if not 1 <= len(scans) <= MAX_SCANS:
        raise ValueError(f"1..{MAX_SCANS} scans per call")
    arr = (CScan * len(scans))(*[s.struct() for s in scans])
    off = [0]
    for n in poses_per_scan:
        off.append(off[-1] + int(n))
    offs = (ctypes.c_int32 * len(off))(*off)
    return arr, offs, off[-1]


def _align(name, mesh, scans, poses_per_scan, T_wc, eps, out, color_tol=0.0):
    dev = mesh.xyz.device
    if isinstance(scans, Scan):
        scans = [scans]
    if poses_per_scan is None:
        poses_per_scan = [T_wc.reshape(-1, 12).shape[0]]
    arr, offs, P = _scan_args(scans, poses_per_scan)
    T = _poses(T_wc, dev)
    if T.shape[0] != P:
        raise ValueError(f"{T.shape[0]} poses given, pose counts sum to {P}")
    if out is None:
        out = torch.empty((P, OUT_STRIDE), dtype=torch.float64, device=dev)
    else:
        _need(out, torch.float64, "out", dev)
        if tuple(out.shape) != (P, OUT_STRIDE):
            raise ValueError("out must be [P, 48]")
    m = mesh.struct()
    context(dev).call(name, ctypes.byref(m), arr, len(scans), ctypes.cast(offs, ctypes.c_void_p), _ptr(T),
                      CCostParams(eps, 0, color_tol), _ptr(out))
    return out


def align_cost(mesh, scans, T_wc, eps=0.1, poses_per_scan=None, out=None, color_tol=0.0):
    """rm_align_cost: [P, 48] result records (E_table, E_soft, counts, ...;
    the color counts when the mesh and the scans carry colors)."""
    return _align("rm_align_cost", mesh, scans, poses_per_scan, T_wc, eps, out, color_tol)


def align_cost_grad(mesh, scans, T_wc, eps=0.1, poses_per_scan=None, out=None, color_tol=0.0):
    """rm_align_cost_grad: as align_cost plus gradient and Gauss-Newton blocks."""
    return _align("rm_align_cost_grad", mesh, scans, poses_per_scan, T_wc, eps, out, color_tol)


def _records(out, P, dev):
    _need(out, torch.float64, "out", dev)
    if tuple(out.shape) != (P, OUT_STRIDE):
        raise ValueError(f"out must be [{P}, {OUT_STRIDE}], got {tuple(out.shape)}")
    return out


def _pose_count(T_wc):
    if T_wc.numel() % 12 or T_wc.shape[-1] not in (4, 12):
        raise ValueError(f"T_wc must hold [P, 12] (or [P, 3, 4]) poses, got {tuple(T_wc.shape)}")
    return T_wc.numel() // 12


def _per_pose(t, P, n, dtype, name, dev):
    _need(t, dtype, name, dev)
    if tuple(t.shape) != (P, n):
        raise ValueError(f"{name} must be [{P}, {n}], got {tuple(t.shape)}")
    return t


def align_cost_grad_noalloc(mesh, scans, T_wc, out, eps=0.1, poses_per_scan=None, color_tol=0.0):
    """rm_align_cost_grad_noalloc: rm_align_cost_grad with its scratch in the
    library's fixed device array (no allocation by the library); `out`
    ([P, 48] f64) must be given."""
    if out is None:
        raise ValueError("out must be given")
    return _align("rm_align_cost_grad_noalloc", mesh, scans, poses_per_scan, T_wc, eps, out, color_tol)


def gn_step(out: torch.Tensor, T_wc: torch.Tensor, lam: float = 0.0, delta_out=None):
    """rm_gn_step: T_wc <- T_wc exp(-(H + lam diag H)^-1 b), in place."""
    dev = T_wc.device
    T = _need(T_wc, torch.float64, "T_wc", dev)
    P = _pose_count(T)
    _records(out, P, dev)
    if delta_out is not None:
        _per_pose(delta_out, P, 6, torch.float64, "delta_out", dev)
    context(dev).call("rm_gn_step", _ptr(out), P, float(lam), _ptr(T), _ptr(delta_out))
    return T_wc


def adam_step(out: torch.Tensor, T_wc: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999):
    """rm_adam_step: Adam on the se(3) increment from the GRAD field; T_wc, m, v in place."""
    dev = T_wc.device
    T = _need(T_wc, torch.float64, "T_wc", dev)
    P = _pose_count(T)
    _records(out, P, dev)
    _per_pose(m, P, 6, torch.float64, "m", dev)
    _per_pose(v, P, 6, torch.float64, "v", dev)
    context(dev).call("rm_adam_step", _ptr(out), P, float(lr), float(beta1), float(beta2), int(step), _ptr(m),
                      _ptr(v), _ptr(T))
    return T_wc


def se3_retract(T_wc: torch.Tensor, delta: torch.Tensor, out=None):
    """rm_se3_retract: T_wc exp(delta) for every pose."""
    dev = T_wc.device
    T = _poses(T_wc, dev)
    P = T.shape[0]
    d = _per_pose(delta.contiguous(), P, 6, torch.float64, "delta", dev)
    o = torch.empty_like(T) if out is None else out
    _need(o, torch.float64, "out", dev)
    if o.numel() != 12 * P:
        raise ValueError(f"out must hold {P} poses of 12 doubles, got {tuple(o.shape)}")
    context(dev).call("rm_se3_retract", _ptr(T), _ptr(d), P, _ptr(o))
    return o


# ---------------------------------------------------------------------------- graphs

class Graph:
    """A captured sequence of library calls (hipGraph), replayed on the
    current stream.  Every call must have run once before capture so that
    the library's scratch is already sized."""

    def __init__(self, device=None):
        self.ctx = context(device)
        self.exec = None

    def __enter__(self):
        self.stream = torch.cuda.Stream(self.ctx.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.ctx.device))
        self._sc = torch.cuda.stream(self.stream)
        self._sc.__enter__()
        self.ctx.lib.rm_ctx_set_stream(self.ctx.handle, ctypes.c_void_p(self.stream.cuda_stream))
        _check(self.ctx.lib.rm_graph_begin(self.ctx.handle), self.ctx.handle)
        return self

    def __exit__(self, *exc):
        h = ctypes.c_void_p()
        rc = self.ctx.lib.rm_graph_end(self.ctx.handle, ctypes.byref(h))
        self._sc.__exit__(*exc)
        torch.cuda.current_stream(self.ctx.device).wait_stream(self.stream)
        if exc[0] is None:
            _check(rc, self.ctx.handle)
            self.exec = h
        return False

    def replay(self):
        self.ctx.lib.rm_ctx_set_stream(self.ctx.handle,
                                       ctypes.c_void_p(torch.cuda.current_stream(self.ctx.device).cuda_stream))
        _check(self.ctx.lib.rm_graph_launch(self.ctx.handle, self.exec), self.ctx.handle)

    def __del__(self):
        try:
            if self.exec is not None and self.exec.value:
                self.ctx.lib.rm_graph_destroy(self.exec)
        except Exception:
            pass


# ---------------------------------------------------------------------------- autograd

class AlignCost(torch.autograd.Function):
    """E_soft(T0 exp(delta)) per pose, differentiable in delta at delta = 0.

    forward(delta [B,6] f64, T0 [B,12] f64, mesh, scan, eps) -> [B] f64.
    The gradient returned is the se(3) gradient of E_soft at T0 exp(delta)
    (exact at delta = 0, where optimizers re-linearize)."""

    @staticmethod
    def forward(ctx, delta, T0, mesh, scan, eps=0.1):
        T = se3_retract(T0, delta.detach())
        out = align_cost_grad(mesh, scan, T, eps)
        ctx.save_for_backward(out[:, OUT_GRAD:OUT_GRAD + 6].clone())
        return out[:, OUT_E_SOFT].clone()

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[:, None] * g, None, None, None, None


# ---------------------------------------------------------------------------- render-accelerated ICP (Sec. V)

def downsample_camera(cam, factor: int = 2):
    """Intrinsics of rm_depth_downsample's output: pixel (u', v') is (factor u', factor v')."""
    from dataclasses import replace
    return replace(cam, fx=cam.fx / factor, fy=cam.fy / factor, cx=cam.cx / factor, cy=cam.cy / factor,
                   width=-(-int(cam.width) // factor), height=-(-int(cam.height) // factor))


def depth_downsample(depth: torch.Tensor, factor: int = 2, z_max: float = 8.0) -> torch.Tensor:
    """rm_depth_downsample: every factor-th pixel of every factor-th row, NaN
    where not a finite positive depth up to z_max."""
    _need(depth, torch.float32, "depth", None)
    H, W = depth.shape
    out = torch.empty((-(-H // factor), -(-W // factor)), dtype=torch.float32, device=depth.device)
    context(depth.device).call("rm_depth_downsample", _ptr(depth), H, W, factor, z_max, _ptr(out))
    return out


def depth_normals(depth: torch.Tensor, cam, sigma: float = 1.0, radius: int = 2) -> torch.Tensor:
    """rm_depth_normals: camera-frame unit normals [H, W, 3] of Eq. (2)."""
    _need(depth, torch.float32, "depth", None)
    H, W = depth.shape
    if (H, W) != (int(cam.height), int(cam.width)):
        raise ValueError("depth must match the camera")
    out = torch.empty((H, W, 3), dtype=torch.float32, device=depth.device)
    context(depth.device).call("rm_depth_normals", _ptr(depth), H, W, float(cam.fx), float(cam.fy), sigma, radius,
                               _ptr(out))
    return out


def vertex_normals(normals: torch.Tensor, stride: int, T_wc) -> torch.Tensor:
    """rm_vertex_normals: world-frame normal of every vertex of the
    rm_mesh_from_range mesh of the same image, stride and pose."""
    _need(normals, torch.float32, "normals", None)
    H, W, _ = normals.shape
    out = torch.empty((-(-H // stride) * -(-W // stride), 3), dtype=torch.float32, device=normals.device)
    keep, pp = _pose_host(T_wc)
    context(normals.device).call("rm_vertex_normals", _ptr(normals), H, W, stride, pp, _ptr(out))
    return out


def icp_cost_grad(mesh, scans, T_wc, vertex_normals: torch.Tensor, tol: float = 0.1, poses_per_scan=None,
                  out=None):
    """rm_icp_cost_grad: [P, 48] ICP records (OUT_ICP_* and the JTR/JTJ blocks)."""
    dev = mesh.xyz.device
    _need(vertex_normals, torch.float32, "vertex_normals", dev)
    if tuple(vertex_normals.shape) != (mesh.xyz.shape[0], 3):
        raise ValueError("vertex_normals must be [n_vertices, 3]")
    if isinstance(scans, Scan):
        scans = [scans]
    if poses_per_scan is None:
        poses_per_scan = [T_wc.reshape(-1, 12).shape[0]]
    arr, offs, P = _scan_args(scans, poses_per_scan)
    T = _poses(T_wc, dev)
    if T.shape[0] != P:
        raise ValueError(f"{T.shape[0]} poses given, pose counts sum to {P}")
    if out is None:
        out = torch.empty((P, OUT_STRIDE), dtype=torch.float64, device=dev)
    else:
        _need(out, torch.float64, "out", dev)
        if tuple(out.shape) != (P, OUT_STRIDE):
            raise ValueError("out must be [P, 48]")
    m = mesh.struct()
    context(dev).call("rm_icp_cost_grad", ctypes.byref(m), _ptr(vertex_normals), arr, len(scans),
                      ctypes.cast(offs, ctypes.c_void_p), _ptr(T), float(tol), _ptr(out))
    return out


def table_cost_weighted(out: torch.Tensor, weights=TABLE_WEIGHTS) -> torch.Tensor:
    """rm_table_cost_weighted: [P] f64 cost sum_k w_k counts_k of result
    records: nine Table I cell weights, optionally followed by the weights of
    the color reward and penalty counts (zero when only nine are given)."""
    import numpy as np
    dev = out.device
    _need(out, torch.float64, "out", dev)
    w = np.asarray(weights, dtype=np.float64).reshape(-1)
    if w.size == 9:
        w = np.concatenate([w, [0.0, 0.0]])
    if w.size != N_WEIGHTS:
        raise ValueError(f"weights must hold 9 or {N_WEIGHTS} values")
    w = np.ascontiguousarray(w)
    P = out.reshape(-1, OUT_STRIDE).shape[0]
    cost = torch.empty(P, dtype=torch.float64, device=dev)
    context(dev).call("rm_table_cost_weighted", _ptr(out), P, w.ctypes.data_as(ctypes.c_void_p), _ptr(cost))
    return cost
