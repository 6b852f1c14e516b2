"""Host-side checks of bench.py's command-line contract and its roofline
arithmetic (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_exits():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2


@pytest.mark.parametrize("n,d,w", [(5, 4, 364), (8, 4, 2628), (8, 6, 3942)])
def test_work_per_amplitude_matches_the_split_counts(n, d, w):
    """W = d (6 C(n,3) + 4 C(n,4) + 2 R + 1) with R = (n-1)(n-2)/2 - 1: the
    three-gluon and four-gluon split counts of the recursion and the
    propagator dots, per field multiply-add."""
    assert bench.work_per_amplitude(n, d) == w
