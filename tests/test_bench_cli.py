"""bench.py's command line on the CPU: a run on more than one GPU is refused
with a message (the solver has a single-GPU path), and the operator-unit and
vector-byte model of the roofline adds up as documented."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_byte_model():
    info = {"iters": 9, "k0": 4, "k1": 3, "cg_iters": 30, "backtracks": 2}
    # 30 CG iterations + 1 per linear step (10 u steps + 5 d steps), less a
    # half per u step prestarted after a K1 step (3), + 10 termination checks
    assert bench.op_units(info) == 30 + 15 - 0.5 * 3 + 10
    n, m, nnz = 20, 50, 100
    per_spmv = nnz * 12 + 4 * (m + 1) + 8 * (m + n)
    assert bench.spmv_bytes(nnz, m, n) == per_spmv
    assert bench.cg_op_bytes(nnz, m, n) == per_spmv + (nnz * 12 + 4 * (n + 1) + 8 * (n + m)) + 10 * n * 8
    N = n + m + 1
    # 18 N-vectors per iteration (projection 5, Anderson 13 for memory 5) and
    # 5 per line-search trial (5 non-K0 iterations + 2 backtracks)
    assert bench.outer_vector_bytes(info, N) == 8.0 * N * (18 * 10 + 5 * 7)
