"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and a non-zero exit, and the algorithmic byte counts
the roofline it reports rests on are the documented ones."""
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
    assert bench.algorithmic_bytes("transport", "p64", "table") == 72
    assert bench.algorithmic_bytes("implicit", "p64", "table") == 168


def test_form_table():
    """Every timed form names a precision and a step kind, and the small
    workloads it times build with the documented shapes."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2606_26268_amd import inputs as I
    table = bench.form_table(I)
    assert {"c3_f32_table", "c3_p64_table", "c1_f32_const", "c1_p64_const", "c2_f32_const", "c2_p64_const",
            "c1_mg8_f32", "c1_mg8_p64", "c3_f32_table_rk2", "c1_mg8_f32_rk2", "c1_f32_general",
            "p0_pulse_f32_rk2", "p0_pulse_p64_rk2"} <= set(table)
    for name, (mk, prec, rk2) in table.items():
        assert prec in ("f32", "p64") and rk2 in (True, False), name
        assert prec in name and (rk2 == name.endswith("_rk2")), name
    g = table["c1_f32_general"][0]()
    assert (g.recon, g.riemann) == (2, 1) and g.bc[0] == [I.REFLECT, I.REFLECT] and g.irr is not None
    assert g.shape == (128, 128, 128)
