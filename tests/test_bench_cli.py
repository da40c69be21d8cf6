"""Host-side checks of bench.py's command line: requests it cannot honour are
refused before anything touches a GPU."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def _run(*args):
    return subprocess.run([sys.executable, str(ROOT / "bench.py"), *args], capture_output=True, text=True,
                          timeout=60)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_unknown_workload_is_refused():
    r = _run("--configs", "kinect,nosuch")
    assert r.returncode == 2
    assert "nosuch" in r.stderr
