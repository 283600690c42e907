"""bench.py host logic: more than one GPU is refused with a message (no
multi-GPU path), bad tuning values are argument errors, and the roofline
constants follow from the method's counts and the chip's unit counts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bad_key_switching_group_size_is_rejected():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--ks-gates-per-block", "8"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "invalid choice" in r.stderr
    assert r.stdout == ""


def test_roofline_constants():
    """The algorithmic count per blind rotation and the derived peak, from
    first principles: 630 CMux steps of 6 forward and 2 inverse 1024-point
    transforms (512 butterflies per stage, 10 stages) plus 2 x 6 pointwise
    rows of 1,024 products; 256 CUs x 64 lanes x 2.4 GHz over 10 VALU
    instructions per modular multiplication (two 5-instruction residue
    butterflies)."""
    sys.path.insert(0, ROOT)
    import bench
    butterflies = (6 + 2) * 10 * 512
    products = 2 * 6 * 1024
    assert bench.MODMUL_PER_BR == 630 * (butterflies + products) == 33_546_240
    assert abs(bench.PEAK_MODMUL - 256 * 64 * 2.4e9 / 10) < 1.0
    assert bench.TRAFFIC_MEASURED["launch"] == {"br_waves_per_rotation": 0, "br_rotations_per_block": 4,
                                                "br_blocks_per_cu": 1, "ks_gates_per_block": 512}
