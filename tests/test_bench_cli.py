"""bench.py's contract that needs no GPU: more than one GPU is refused with a message, and
the interior kernel's algorithmic bytes per cell-update are the compulsory read and write
of the stored planes."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_cell_update():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.ALG_BYTES == {"f64": 2 * 33 * 8, "f32": 2 * 33 * 4, "f32dev": 2 * (33 * 4 + 4 * 8)}
    assert bench.HBM_PEAK_GBS == 8000.0
