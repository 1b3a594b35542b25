"""CPU checks of bench.py's host logic: the single-GPU guard and the
algorithmic-bytes model's parts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_algorithmic_bytes_parts():
    sys.path.insert(0, ROOT)
    import bench
    n, E, d, esz = 1000, 3000, 10, 4
    base = bench.algorithmic_bytes(n, E, d, esz, 0, 0, 1, 1)
    # one CG iteration adds the slot data, row pointers, diagonal and ten n x d streams
    one_it = bench.algorithmic_bytes(n, E, d, esz, 1, 1, 1, 1) - base
    assert one_it == 16 * E + 4 * (n + 1) + 2 * n * esz + 10 * n * d * esz
    # without the P/B update the Gram and apply passes (2n + 6nd values) drop out
    assert base - bench.algorithmic_bytes(n, E, d, esz, 0, 0, 1, 1, pupdate=False) == 2 * n * esz + 6 * n * d * esz
    # each further inner step adds the edge update with b read and written per edge
    step = bench.algorithmic_bytes(n, E, d, esz, 0, 0, 2, 1) - base
    assert step == 16 * E + 4 * (n + 1) + 3 * n * esz + 4 * n * d * esz + 2 * E * d * esz + 4 * E
