"""Host-side checks of bench.py (no GPU): the script parses and imports, its byte
model covers the kernels of each preconditioner layout, the stored counter
traffic belongs to the committed dense-solve source, and a multi-GPU request
exits with a message."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_kernel_bytes_per_layout():
    b = _bench()
    info = {"n_free": 1000, "sum_np": 1500, "n_jent": 1300}
    # reduced system on the local systems' stream: phase 1 carries the J^T stage
    kb = b.kernel_bytes(dict(info, reduced_stream=0, local_iters=0), 900, "fp64")
    assert kb["R_p+J^T"] == 1300 * (4 + 8 + 3 * 8 + 8)
    assert kb["x,r update"] == 1000 * 48
    assert kb["A+p"] == 900 * (224 + 16) + 1000 * 32
    # reduced branch on the second stream with stored inverses: nothing in phase 1
    kb = b.kernel_bytes(dict(info, reduced_stream=1, local_iters=0), 900, "mixed")
    assert "R_p+J^T" not in kb
    # inexact local solves: phase 1 is the R_p gather
    kb = b.kernel_bytes(dict(info, reduced_stream=1, local_iters=8), 900, "mixed")
    assert kb["R_p+J^T"] == 1500 * (4 + 8 + 4)


def test_stored_traffic_matches_the_committed_gemv_source():
    b = _bench()
    t = b.GEMV_TRAFFIC["annulus128"]
    assert b._traffic("annulus128") == t["bytes"]
    # the bytes follow from the stored counter readings (scales rounded to 2.0 and 1.0)
    est = t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"]
    assert abs(t["bytes"] - est) < 1e-4 * est


def test_multi_gpu_request_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in p.stdout + p.stderr
