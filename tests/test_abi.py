"""CPU checks of the C ABI boundary: the built library loads, exports every
function include/rendermap.h declares, and rejects invalid arguments on the
host before touching a device.  No compute call runs here."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "rendermap.h"
LIB = ROOT / "paper_1702_06813_amd" / "librendermap.so"


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(rm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        pytest.skip("library not built")
    return ctypes.CDLL(str(LIB))


def test_header_declares_the_boundary():
    names = declared_functions()
    for core in ("rm_mesh_from_range", "rm_render_depth", "rm_align_cost", "rm_align_cost_grad"):
        assert core in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_symbol_list_matches_header():
    from paper_1702_06813_amd import rendermap
    assert sorted(rendermap.ABI_SYMBOLS) == declared_functions()


def test_null_context_is_rejected_without_a_device(lib):
    lib.rm_last_error.restype = ctypes.c_char_p
    lib.rm_last_error.argtypes = [ctypes.c_void_p]
    assert lib.rm_render_depth(None, None, None, None, 0, None, None, None) == -1
    assert b"ctx" in lib.rm_last_error(None)
    assert lib.rm_gn_step(None, None, 1, ctypes.c_double(0.0), None, None) == -1
    from paper_1702_06813_amd.rendermap import CCostParams
    fn = lib.rm_align_cost
    fn.argtypes = [ctypes.c_void_p] * 6 + [CCostParams, ctypes.c_void_p]
    assert fn(None, None, None, 1, None, None, CCostParams(0.1, 0, 0.0), None) == -1


def test_cluster_size_rule(lib):
    lib.rm_mesh_clusters_size.restype = ctypes.c_int64
    lib.rm_mesh_clusters_size.argtypes = [ctypes.c_int64]
    # [ceil(T/256)] 32-byte cluster records padded to 256 bytes, then [T][3] f32 normals
    assert lib.rm_mesh_clusters_size(0) == 0
    for T in (1, 256, 257, 2048, 2049, 1021734):
        C = -(-T // 256)
        assert lib.rm_mesh_clusters_size(T) == (C * 32 + 255) // 256 * 256 + 12 * T


def test_ctx_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = lib.rm_ctx_create(0, ctypes.byref(h))
    assert rc in (-3, -1) and not h.value


def test_product_path_does_not_use_the_oracle():
    """The package never imports, loads or names the oracle."""
    pkg = ROOT / "paper_1702_06813_amd"
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + list(pkg.rglob("*.cpp")) + list(pkg.rglob("*.h")):
        text = f.read_text()
        assert "oracle" not in text.lower(), f
        assert "rm_oracle" not in text, f


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1702_06813_amd as rm
    with pytest.raises(RuntimeError):
        rm.Context(0)


def test_microbenchmark_library_exports_and_rejects_bad_arguments():
    """The atomic-throughput microbenchmarks the benchmark reports beside the
    roofline: both symbols exported, out-of-range arguments rejected (-1)
    before any device call."""
    path = ROOT / "paper_1702_06813_amd" / "librm_microbench.so"
    if not path.exists():
        pytest.skip("microbenchmark library not built")
    mb = ctypes.CDLL(str(path))
    dp = ctypes.POINTER(ctypes.c_double)
    mb.rm_mb_lds_min_u64.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    mb.rm_mb_global_atomic_add.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    s, n = ctypes.c_double(), ctypes.c_double()
    assert mb.rm_mb_lds_min_u64(0, 8, ctypes.byref(s), ctypes.byref(n)) == -1
    assert mb.rm_mb_lds_min_u64(16, 0, ctypes.byref(s), ctypes.byref(n)) == -1
    assert mb.rm_mb_global_atomic_add(16, 8, 5, ctypes.byref(s), ctypes.byref(n)) == -1
    assert mb.rm_mb_global_atomic_add(16, 8, 25, ctypes.byref(s), ctypes.byref(n)) == -1
    assert mb.rm_mb_global_atomic_add(16, 8, 12, None, ctypes.byref(n)) == -1


def test_struct_layouts_match_the_binding(tmp_path):
    """sizeof and offsetof of the ABI structs, as a C compiler lays them out
    from the header, equal the binding's ctypes mirrors."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    from paper_1702_06813_amd import rendermap as R
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", str(ROOT / "include"), "-o", str(exe),
                    str(ROOT / "tests" / "native" / "abi_layout.c")], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                               check=True).stdout.splitlines())
    mirrors = {"rm_camera": R.CCamera, "rm_mesh": R.CMesh, "rm_scan": R.CScan, "rm_cost_params": R.CCostParams}
    for name, cls in mirrors.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for key, val in got.items():
            if key.startswith(name + "."):
                assert getattr(cls, key.split(".", 1)[1]).offset == int(val), key
