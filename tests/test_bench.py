"""bench.py's host-side bookkeeping, on the CPU: the --gpus guard, the
whole-solve fraction and the P2P kernel named in the roofline."""
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_solve_fraction_sums_phase_ideals():
    args = types.SimpleNamespace(n=1_000_000)
    work = {"far": 78.6e9, "near": 2 * 78.6e9}  # 1 ms and 2 ms at the FP64 peak
    f = bench.solve_fraction(args, work, 10.0)
    assert abs(f["ideal_ms"]["far"] - 1.0) < 1e-9
    assert abs(f["ideal_ms"]["near"] - 2.0) < 1e-9
    tree = 1e6 * bench.TREE_BYTES_PER_PARTICLE / 8e12 * 1e3
    assert abs(f["ideal_ms"]["tree"] - round(tree, 4)) < 1e-9
    assert abs(f["frac"] - round((3.0 + tree) / 10.0, 4)) < 1e-9


def test_near_shape_names_the_launched_kernel():
    # the roofline's kernel name follows the near-kernel number and leaf size
    # the same way the C++ dispatch does
    assert bench.near_shape("fp64", 10, 0) == "near"
    assert bench.near_shape("fp64", 10, 7) == "near"
    assert bench.near_shape("fp64", 10, 1) == "near_thread"
    assert bench.near_shape("fp64", 10, 6) == "near_leaf"
    assert bench.near_shape("fp64", 10, 13) == "near_tile"
    assert bench.near_shape("fp64", 16, 0) == "near"
    assert bench.near_shape("fp64", 16, 6) == "near_leaf"
    assert bench.near_shape("fp64", 24, 0) == "near"
    assert bench.near_shape("fp64", 32, 13) == "near_tile"
    assert bench.near_shape("fp64", 40, 0) == "near_thread"
    assert bench.near_shape("fp32c", 10, 0) == "near"
    assert bench.near_shape("fp32c", 10, 7) == "near"
    assert bench.near_shape("fp32c", 10, 6) == "near_leaf"
    for prec in ("fp64", "fp32c"):
        for ls in (10, 16, 24, 40):
            for v in (0, 1, 6, 7, 13):
                assert (prec, bench.near_shape(prec, ls, v)) in bench.KERNELS
