"""Host-side checks of bench.py: the one-GPU contract and the algorithmic-byte
count the roofline fraction divides by."""
import os
import subprocess
import sys

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_bench_workload():
    """48^3 N1curl2, FP32 inverses, one column: x and y (8 n each), the map
    (4 n_br) and the packed lower triangles (4 * 210 per element)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    w = workloads.BY_NAME["n1curl2_3d_48_jit"]
    n, E, nl = 4271904, 663552, 20
    expect = 8 * n + 8 * n + 4 * E * nl + 4 * E * nl * (nl + 1) // 2
    assert b.algorithmic_bytes(w, n, E, nl, 1, w.prec) == expect == 678818304
