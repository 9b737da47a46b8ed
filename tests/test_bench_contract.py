"""The command-line contract of bench.py, checked without a GPU: the flags
the benchmark is driven with, and the refusal of more than one GPU (the path
runs on a single MI355X; sharding is described, not built)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_help_lists_the_driving_flags():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--only", "--mixed-radix-only", "--copy-calibration"):
        assert flag in r.stdout


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = _run("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "single MI355X" in r.stderr
    assert r.stdout.strip() == ""


def test_kernel_hash_covers_the_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.kernel_hash()
    assert len(h) == 16 and int(h, 16) >= 0
