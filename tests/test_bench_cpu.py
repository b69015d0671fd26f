"""Host-side parts of the benchmark: the algorithmic byte counts of the
measured workload (the figures the roofline is computed from), the vector
peak it is compared with, and the one-GPU guard of the command line."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_benchmark_workload():
    import bench
    n_p, gpd, step = bench.algorithmic_bytes(bench.workload())
    # 256^3 cells, slab of 256 x 256 x 26 cells at 2 x 8 particles per cell
    assert n_p == 256 * 256 * 26 * 16 == 27_262_976
    P = 4
    occ = 256 * 256 * 26
    assert gpd == n_p * 13 * P + occ * 9 * P == 1_479_016_448
    assert step == gpd + 256 ** 3 * 15 * P
    # 91.2 bytes per particle-step
    assert abs(step / n_p - 91.2) < 0.05


def test_vector_peaks():
    import bench
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz, and twice that with
    # packed instructions (the published 157.3 TFLOP/s)
    assert abs(bench.FP32_VECTOR_PEAK_TFS - 78.6) < 0.1
    assert abs(bench.FP32_PACKED_PEAK_TFS - 157.3) < 0.1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_host_cores_and_one_oracle_sample():
    import bench
    avail, workers = bench.host_cores()
    assert 1 <= workers <= min(16, avail)
    # one sample step of the all-core oracle timing (its per-process unit)
    n, t_step, t_yee = bench._oracle_sample_step((500, 1, 4))
    assert n == 1000 and t_step > t_yee > 0
