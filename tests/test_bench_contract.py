"""bench.py's contract pieces that need no GPU: a multi-GPU request exits
with a message (one GPU only), and the algorithmic byte model behind the
roofline fraction counts 80 Np bytes of FP32 state traffic per element-stage
plus the geometry the running kernel reads (FP32 tiles: 100 B; FP64: 200 B)
and 20 B of connectivity."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_byte_model():
    b = _bench()
    for Np in (10, 20, 35, 56):
        assert b.stage_bytes(1, Np, True, 0) == 80 * Np + 120
        assert b.stage_bytes(1, Np, True, 1) == 80 * Np + 220
        assert b.stage_bytes(1, Np, False, 0) == 60 * Np + 120
    # the c2 workload: 207,900 tets at N = 4
    assert b.stage_bytes(207_900, 35, True, 0) == 607_068_000
    assert b.stage_bytes(207_900, 35, True, 1) == 627_858_000
