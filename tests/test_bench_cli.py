"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and a non-zero exit, and the algorithmic byte and
operation counts it reports are the documented ones."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_documented_counts():
    sys.path.insert(0, ROOT)
    import bench
    # bytes per cell: transport 9 fields, implicit 8 radiation + 9 gas doubles, + cache
    assert bench.algorithmic_bytes("transport", "f32", "mlp") == 36
    assert bench.algorithmic_bytes("implicit", "f32", "mlp") == 120
    assert bench.algorithmic_bytes("implicit", "p64", "const") == 136
    assert bench.algorithmic_valu_ops("implicit", "mlp") == 1250
    assert bench.algorithmic_valu_ops("transport", "mlp") == 696
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
