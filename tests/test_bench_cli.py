"""The benchmark's command line on the CPU: it measures one GPU and says so
when asked for more (the multi-GPU sweep is not implemented)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_paper_flop_model_counts():
    """The paper's count (Sec. V-A): per subject two v x t x k products
    (2 v t k flops each), one v x k x k product and an economy SVD counted as
    Householder QR, 2 m n^2 - 2 n^3 / 3; additive over subjects."""
    import bench
    one = bench.paper_flop_model([1000], 200, 10)
    assert one == 2 * (2 * 1000 * 200 * 10) + 2 * 1000 * 10 * 10 + (2 * 1000 * 100 - 2 * 1000 / 3)
    assert abs(bench.paper_flop_model([1000, 3000], 200, 10)
               - bench.paper_flop_model([1000], 200, 10)
               - bench.paper_flop_model([3000], 200, 10)) < 1e-6
