"""Host-side checks of bench.py (no GPU): the one-GPU guard and the
algorithmic byte counts of the roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    n, k = 1 << 24, 838_861
    # mask once, records read (32 B) and slots written (32 B) per update
    assert bench.algorithmic_bytes("select_update", n, k) == n + 64 * k
    # alive read everywhere, alive set, records read and slots written
    assert bench.algorithmic_bytes("add_agents", n, k) == 4 * n + 68 * k
    # mask once, alive read and written where killed
    assert bench.algorithmic_bytes("remove_agents", n, k) == n + 8 * k
    with pytest.raises(ValueError):
        bench.algorithmic_bytes("sort", n, k)


def test_median_helper():
    assert bench._med([3.0, 1.0, 2.0]) == 2.0
    assert bench._med([5.0]) == 5.0


def test_cpu_model_string_is_read():
    assert isinstance(bench._cpu_model(), str) and bench._cpu_model()
