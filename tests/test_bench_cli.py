"""bench.py's command line on the host: one GPU only, and the C5 serving defaults (200 measured
requests after 20 warm-up at 90 % of the saturation rate)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_c5_defaults():
    sys.path.insert(0, ROOT)
    import bench

    old = sys.argv
    try:
        sys.argv = ["bench.py", "--workload", "c5"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert (a.c5_count, a.c5_warmup, a.c5_kmax) == (200, 20, 11)
    assert a.c5_loads == "0.9" and not a.c5_compare and a.c5_qps == "auto"
    assert (a.c5_max_running, a.c5_piece, a.c5_busy_running, a.c5_lanes) == (2, 5, 1, 0)
