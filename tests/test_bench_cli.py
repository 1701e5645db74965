"""bench.py's command-line contract that needs no GPU: asking for more than
one GPU, or a precision outside the graded-only measurement, ends with a
message and exit status 2 before any device work."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2", "--steps", "1", "--warmup", "0"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_dtype_needs_graded_only():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--dtype", "f64"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--graded-only" in r.stderr
    assert r.stdout.strip() == ""
