"""Host-side checks of the benchmark script: the one-GPU guard and the
algorithmic flop count its headline divides by (the block build of Eq. 3 on
the one-block basis: H_b full and S_b's upper triangle, d_b = 1 + M_b +
N_O (N_B - 1) with the Theta columns of the other blocks, Eq. 9-10)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


def test_build_flops_of_the_4096_parameter_workload():
    import bench
    # 8 blocks of 512 parameters, one previous direction: d = 1 + 512 + 7 = 520
    # per pencil; 2 N_s (d^2 + d (d + 1) / 2) per block
    offsets = [512 * b for b in range(9)]
    fl = bench.build_flops(offsets, 1, 1_000_000)
    assert fl == 2 * 1_000_000 * 8 * (520 * 520 + 520 * 521 // 2)
    assert fl == pytest.approx(6.49376e12, rel=1e-12)


def test_build_flops_counts_every_block_with_its_own_width():
    import bench
    # uneven blocks, no previous directions: d = 1 + M_b
    offsets = [0, 3, 10, 11]
    want = sum((1 + m) ** 2 + (1 + m) * (2 + m) / 2 for m in (3, 7, 1))
    assert bench.build_flops(offsets, 0, 5) == 2 * 5 * want
    # with two previous directions each block also carries 2 (N_B - 1) = 4 Theta columns
    want2 = sum((5 + m) ** 2 + (5 + m) * (6 + m) / 2 for m in (3, 7, 1))
    assert bench.build_flops(offsets, 2, 5) == 2 * 5 * want2
