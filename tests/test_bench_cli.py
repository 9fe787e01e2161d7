"""The benchmark's command-line contract on the CPU: more than one GPU is
refused with a JSON error line before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "--gpus must be 1" in line["error"]


def test_bench_screen_families_map_to_the_library_options():
    """Every --screen choice names a (support, q) pair the library accepts:
    the one-element screens of degree 2..4 and the 27-element screens of
    degree 1..4, with the method's default first in the help."""
    sys.path.insert(0, ROOT)
    import bench

    assert bench.SCREENS["one-q3"] == ("one", 3)
    assert sorted(bench.SCREENS.values()) == sorted([("one", 2), ("one", 3), ("one", 4),
                                                      ("27", 1), ("27", 2), ("27", 3), ("27", 4)])
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--screen", "27-q5"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2 and "invalid choice" in r.stderr
