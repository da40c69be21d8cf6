"""The FP64 oracle's C source built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) renders the tiny room and a
ragged meshified view without a report, and every output equals the
shared-library build bit for bit.  CPU only."""
import os
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

from workloads import configs, scenes as S

ROOT = Path(__file__).resolve().parent.parent
DRIVER = Path(__file__).resolve().parent / "native" / "oracle_asan_main.c"
ORACLE_C = ROOT / "oracle" / "rm_oracle.c"


@pytest.fixture(scope="module")
def asan_exe(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = tmp_path_factory.mktemp("asan") / "oracle_asan"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-o", str(exe), str(DRIVER), str(ORACLE_C), "-lm"]
    subprocess.run(cmd, check=True)
    return exe


def _request(path, depth, cam, T_map, T_query, stride, radius, z_min, z_max, max_edge):
    H, W = depth.shape
    with open(path, "wb") as f:
        f.write(np.array([H, W], np.int32).tobytes())
        f.write(np.array([cam.fx, cam.fy, cam.cx, cam.cy], np.float32).tobytes())
        f.write(np.array([cam.width, cam.height], np.int32).tobytes())
        f.write(np.array([cam.z_near, cam.z_far], np.float32).tobytes())
        f.write(np.ascontiguousarray(T_map, np.float64).reshape(12).tobytes())
        f.write(np.ascontiguousarray(T_query, np.float64).reshape(12).tobytes())
        f.write(np.array([stride, radius], np.int32).tobytes())
        f.write(np.array([z_min, z_max, max_edge], np.float32).tobytes())
        f.write(np.ascontiguousarray(depth, np.float32).tobytes())


class _Reader:
    def __init__(self, data):
        self.b, self.o = data, 0

    def take(self, dtype, n):
        a = np.frombuffer(self.b, dtype, count=n, offset=self.o)
        self.o += a.nbytes
        return a


def _run(exe, tmp, *args):
    req, rep = tmp / "req.bin", tmp / "rep.bin"
    _request(req, *args)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([str(exe), str(req), str(rep)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return _Reader(rep.read_bytes())


def _compare(oracle_mod, R, depth, cam, T_map, T_query, stride, radius, z_min, z_max, max_edge):
    O = oracle_mod
    H, W = depth.shape
    d_ref, c_ref = O.scan_image(depth, z_min, z_max)
    np.testing.assert_array_equal(R.take(np.float32, H * W).view(np.uint32), d_ref.reshape(-1).view(np.uint32))
    np.testing.assert_array_equal(R.take(np.uint8, H * W), c_ref.reshape(-1))
    xyz, tri, cls = O.meshify(depth, cam, T_map, stride, z_min, z_max, max_edge, radius)
    nv, nt = R.take(np.int64, 2)
    assert (nv, nt) == (xyz.shape[0], tri.shape[0]) and nt > 0
    np.testing.assert_array_equal(R.take(np.float32, 3 * nv).view(np.uint32), xyz.reshape(-1).view(np.uint32))
    np.testing.assert_array_equal(R.take(np.int32, 3 * nt), tri.reshape(-1))
    np.testing.assert_array_equal(R.take(np.uint8, nt), cls)
    n = cam.width * cam.height
    covered = 0
    for mode in ("contract", "exact"):
        ref = O.render((xyz, tri), cam, T_query, mode=mode)
        for key, dt, k in (("z", np.float64, 1), ("id", np.int32, 1), ("z2", np.float64, 1),
                           ("ncov", np.int32, 1), ("nrm", np.float64, 3)):
            got = R.take(dt, k * n)
            want = np.ascontiguousarray(ref[key], dt).reshape(-1)
            if dt == np.float64:
                np.testing.assert_array_equal(got.view(np.uint64), want.view(np.uint64), err_msg=f"{mode} {key}")
            else:
                np.testing.assert_array_equal(got, want, err_msg=f"{mode} {key}")
        assert int(R.take(np.int64, 1)[0]) == ref["dropped"]
        covered += int((ref["id"] >= 0).sum())
    subs = O.contract_subtriangles((xyz, tri), cam, T_query)
    nsub = int(R.take(np.int64, 1)[0])
    assert nsub == len(subs)
    np.testing.assert_array_equal(R.take(np.int64, 7 * nsub).reshape(-1, 7), np.asarray(subs, np.int64).reshape(-1, 7))
    assert R.o == len(R.b)
    return covered


def test_oracle_under_sanitizers_tiny_room(asan_exe, oracle_mod, tmp_path):
    """The tiny room's scan, meshified from its own pose (stride 2, node
    smoothing radius 1), rendered from the candidate pose 5 cm / 2 deg away,
    both coverage modes, full 64x48 frame."""
    w = configs.tiny(0)
    args = (w.scan_depth, w.cam, w.T_true, w.poses[0], 2, 1, w.z_min, w.z_max, 0.1)
    R = _run(asan_exe, tmp_path, *args)
    assert _compare(oracle_mod, R, *args) > 0


def test_oracle_under_sanitizers_ragged_view(asan_exe, oracle_mod, tmp_path):
    """A ragged 37x23 image (stride 3 leaves partial quads at the border) with
    dead and no-return pixels, rendered from a pose that puts part of the
    mesh behind the near plane (contract clipping runs)."""
    cam = S.Camera(20.0, 20.0, 18.0, 11.0, 37, 23, 0.1, 8.0)
    scene = S.random_box_room(3, (4.0, 4.0, 2.5), 6)
    c = 0.5 * (scene.room_lo + scene.room_hi)
    T = S.look_pose(np.array([c[0], c[1], 1.3]), 0.7, 0.1)
    depth = S.range_image(scene, cam, T, 7, noise_rel=0.01, dropout=0.05, dead=0.05)
    T_q = T.copy()
    T_q[:, 3] += T[:, :3] @ np.array([0.0, 0.0, 1.5])       # 1.5 m forward: walls cross the near plane
    args = (depth, cam, T, T_q, 3, 0, 0.5, 8.0, 0.1)
    R = _run(asan_exe, tmp_path, *args)
    assert _compare(oracle_mod, R, *args) > 0
