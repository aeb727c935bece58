"""bench.py's host-side contract: more than one GPU is refused with a
message, and the algorithmic byte counts of the stage kernels."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stage_bytes():
    sys.path.insert(0, ROOT)
    import bench
    # S-stage: 9 FP64 matrix planes + r, v, r_hat read + s, t written = 112 B per unknown (2D)
    assert bench.stage_bytes(1000, 2, 8, 8) == 112_000
    assert bench.stage_bytes(1000, 2, 4, 8) == 76_000
    assert bench.stage_bytes(1000, 3, 8, 8) == 256_000
    # P-stage: 9 planes + 10 vector streams (s, t, p, v, x, rhat read; r, p', x, v' written)
    assert bench.stage_bytes(1000, 2, 8, 8, "P") == 152_000
    assert bench.stage_bytes(1000, 3, 8, 8, "P") == 296_000
    assert bench.stage_bytes(1000, 3, 4, 8, "P") == 188_000
    # the set's own FP64 operator: the off-centre planes (2D: 8) and, in 3D, the 1-byte unknown flag
    assert bench.stage_bytes(1000, 2, 8, 8, "S", True) == 104_000
    assert bench.stage_bytes(1000, 2, 8, 8, "P", True) == 144_000
    assert bench.stage_bytes(1000, 3, 8, 8, "S", True) == 249_000
    assert bench.stage_bytes(1000, 3, 8, 8, "P", True) == 289_000
