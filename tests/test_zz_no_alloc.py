"""GPU test of the allocation-free entry point rm_align_cost_grad_noalloc
against rm_align_cost_grad, through the C ABI: two calls in a row (the
second with a smaller input), a call at the benchmark's shape, and the
rejection of a call whose scratch exceeds the fixed array."""
import sys

import numpy as np
import pytest

from workloads import scenes as S

from gpu_helpers import EPS, oracle_map, workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1702_06813_amd as rm
    rm.load_library()
    return rm


def _T(poses):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(poses).reshape(-1, 12))).to(DEV)


def _case(rm, name, n_poses, tile=None):
    w = workload(name)
    mesh = rm.Mesh.from_arrays(*oracle_map(name), device=DEV).prepare()
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), w.z_min, w.z_max, cam=w.cam)
    T = _T(w.poses[:n_poses])
    return mesh, scan, T


def test_noalloc_matches_align_cost_grad_twice(rm):
    """Kinect-like map, 16 poses, then the tiny room, 1 pose: the fixed-array
    call gives the records of rm_align_cost_grad bit for bit, each time (the
    array keeps the first call's contents; the second call clears what it
    needs)."""
    _say("noalloc: kinect 16 poses, then tiny 1 pose")
    for name, n in (("kinect", 16), ("tiny", 1)):
        mesh, scan, T = _case(rm, name, n)
        ref = rm.align_cost_grad(mesh, scan, T, EPS).cpu().numpy()
        out = torch.full((T.shape[0], rm.OUT_STRIDE), float("nan"), dtype=torch.float64, device=DEV)
        rm.align_cost_grad_noalloc(mesh, scan, T, out, EPS)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        # without prepared clusters the bounds go into the fixed array too
        bare = rm.Mesh(mesh.xyz, mesh.tri, mesh.cls)
        out.fill_(float("nan"))
        rm.align_cost_grad_noalloc(bare, scan, T, out, EPS)
        np.testing.assert_array_equal(out.cpu().numpy(), ref)


@pytest.mark.slow
def test_noalloc_benchmark_shape(rm):
    """The 1M-triangle map with 64 poses: the bins share the fixed array with
    the rest of the scratch; records equal rm_align_cost_grad's."""
    _say("noalloc: differentiation 64 poses")
    mesh, scan, T = _case(rm, "differentiation", 64)
    ref = rm.align_cost_grad(mesh, scan, T, EPS).cpu().numpy()
    out = torch.empty((64, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
    rm.align_cost_grad_noalloc(mesh, scan, T, out, EPS)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


def test_noalloc_rejects_scratch_beyond_the_array(rm):
    """65,535 poses against the Kinect-like map need ~0.6 GB of visible
    cluster lists alone: refused with RM_ERR_CAPACITY before any launch, and
    the next call works."""
    _say("noalloc: oversize request")
    w = workload("kinect")
    mesh = rm.Mesh.from_arrays(*oracle_map("kinect"), device=DEV).prepare()
    scan = rm.scan_image(torch.from_numpy(w.scan_depth).to(DEV), w.z_min, w.z_max, cam=w.cam)
    P = 65535
    T = _T(np.repeat(w.poses[:1], P, axis=0))
    out = torch.zeros((P, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
    with pytest.raises(rm.RenderMapError) as ex:
        rm.align_cost_grad_noalloc(mesh, scan, T, out, EPS)
    assert ex.value.code == rm.RM_ERR_CAPACITY
    assert "allocation-free buffer" in str(ex.value)
    assert not out.any()
    ref = rm.align_cost_grad(mesh, scan, T[:2].contiguous(), EPS).cpu().numpy()
    o2 = torch.empty((2, rm.OUT_STRIDE), dtype=torch.float64, device=DEV)
    rm.align_cost_grad_noalloc(mesh, scan, T[:2].contiguous(), o2, EPS)
    np.testing.assert_array_equal(o2.cpu().numpy(), ref)
