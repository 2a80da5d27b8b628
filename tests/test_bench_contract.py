"""Host checks of bench.py's command-line contract (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_workload_is_rejected():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "invalid choice" in r.stderr


def test_layered_batch_source_list_is_checked_before_any_device_work():
    for bad in ("32", "0-40", "3,3", "x"):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "3d-layered-batch",
                            "--sources", bad], capture_output=True, text=True, timeout=120)
        assert r.returncode == 2, bad
        assert "distinct indices in 0..31" in r.stderr and r.stdout == "", bad
