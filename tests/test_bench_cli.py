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


def test_colella_exact_fixture_is_current(tmp_path):
    """The stored exact Colella solution is what its committed script writes now."""
    import json
    import shutil
    gold = os.path.join(ROOT, "tests", "golden")
    work = tmp_path / "golden"
    work.mkdir()
    shutil.copy(os.path.join(gold, "make_colella_exact.py"), work)
    # the script writes next to itself and imports oracle from two levels up
    script = work / "make_colella_exact.py"
    text = script.read_text().replace("sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))",
                                      f"sys.path.insert(0, {ROOT!r})")
    script.write_text(text)
    subprocess.run([sys.executable, str(script)], check=True, timeout=120)
    a = json.load(open(work / "colella_exact_j4m.json"))
    b = json.load(open(os.path.join(gold, "colella_exact_j4m.json")))
    assert a == b
    assert abs(b["star"]["p"] - 431.3446) < 1e-3 and sum(b["smooth"]) > 800
