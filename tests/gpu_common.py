"""Shared helpers of the GPU parity tests: run a problem through the HIP
library and through the oracle, and compare per field (normwise relative
L1 and L-infinity errors)."""
import sys

import numpy as np

RAD = ("E", "Fx", "Fy", "Fz")
ALL = ("E", "Fx", "Fy", "Fz", "mx", "my", "mz", "Eg")

# float64 form: rounding-level agreement; float32 transport: 1e-5 per field
TOL_P64 = dict(l1=1e-12, linf=1e-10)
TOL_F32 = dict(l1=1e-5, linf=1e-5)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_errors(got, ref, fields=ALL):
    out = {}
    for k in fields:
        d = np.abs(got[k] - ref[k])
        s1 = np.abs(ref[k]).sum()
        sinf = np.abs(ref[k]).max()
        out[k] = (d.sum() / s1 if s1 > 0 else d.sum(), d.max() / sinf if sinf > 0 else d.max())
    return out


def assert_close(got, ref, tol, fields=ALL, label=""):
    errs = rel_errors(got, ref, fields)
    bad = {k: v for k, v in errs.items() if v[0] > tol["l1"] or v[1] > tol["linf"]}
    say(f"  {label} " + " ".join(f"{k}:{v[0]:.1e}/{v[1]:.1e}" for k, v in errs.items()))
    assert not bad, f"{label} parity failed: {bad}"
    return errs


def run_gpu(prob, precision, steps, dt=None, mlp=None):
    from paper_2606_26268_amd import m1
    s = m1.Solver(prob, precision=precision, mlp=mlp)
    s.step(prob.dt if dt is None else dt, steps)
    st = s.state()
    diag = s.diagnostics()
    s.close()
    return st, diag


def run_oracle(orc, prob, steps, dt=None, mlp=None):
    o = orc.Oracle(prob, mlp)
    return o.run(prob.fields, prob.dt if dt is None else dt, steps)
