"""Host-side pieces of bench.py (CPU): the algorithmic bytes the roofline
object divides by the measured time, the VALU issue rate, and the
one-GPU contract of the command line."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_of_the_padded_convolution():
    """Per kernel, counted from the arrays it must touch: K1 reads p (N^2)
    and writes the half spectrum of the N data rows (N x (N + 1) complex);
    K2 reads and writes that half spectrum once and reads the
    (N + 1)^2 quadrant table; K3 reads the half spectrum and writes u."""
    for N, s in [(64, 8), (512, 4), (1024, 4), (1024, 8), (2048, 4)]:
        spec = N * (N + 1) * 2 * s            # complex values of s bytes per part
        b = bench.alg_bytes(N, s)
        assert b["k1_rows_fwd"] == N * N * s + spec
        assert b["k2_cols"] == 2 * spec + (N + 1) ** 2 * s
        assert b["k3_rows_inv"] == spec + N * N * s
        assert b["apply"] == 2 * s * N * N + 8 * s * N * (N + 1) + s * (N + 1) ** 2
    assert bench.alg_bytes(1024, 4)["k2_cols"] == 20996100
    assert bench.alg_bytes(1024, 4)["apply"] == 46178308


def test_valu_issue_rate():
    # 256 CUs x 4 SIMDs, a wave64 instruction every 4 cycles on a 16-lane SIMD, 2.4 GHz
    assert bench.VALU_ISSUE_PER_S == 256 * 4 * 2.4e9 / 4
    assert bench.PEAK_HBM_GBPS == 8000.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
