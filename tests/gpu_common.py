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
# float64 form with states at f = 1 (free-streaming beams, clipped faces): the
# signal speeds depend on sqrt(1 - f) terms, so a rounding change of f moves
# them by ~sqrt(eps64) = 1.5e-8; ten times that, per step count of ~1e2
TOL_P64_F1 = dict(l1=1e-7, linf=1e-6)


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


def assert_close_f32(got, ref, fields=ALL, label="", gas_scale=1.0):
    """FP32 transport vs the FP64 oracle.

    rel-L1 <= 1e-5 per field (radiation; gas fields scaled by gas_scale for
    c >> c_hat, where E_g absorbs (c/c_hat) times the FP32 rounding of E).
    The f-preserving face fix is discontinuous, so rounding-level
    differences flip a few face decisions and the affected cells (whose
    perturbation then spreads at up to c_hat) move by far more than the
    rounding: rel-L-infinity is capped at 1e-2 and the number of cells above
    1e-5 max|ref| is reported.
    """
    errs = rel_errors(got, ref, fields)
    flips = {}
    for k in fields:
        d = np.abs(got[k] - ref[k])
        flips[k] = int((d > 1e-5 * np.abs(ref[k]).max()).sum())
    say(f"  {label} " + " ".join(f"{k}:{v[0]:.1e}/{v[1]:.1e}/{flips[k]}" for k, v in errs.items()))
    bad = {}
    for k, (l1, linf) in errs.items():
        scale = gas_scale if k in ("mx", "my", "mz", "Eg") else 1.0
        if l1 > 1e-5 * scale or linf > 1e-2 * scale:
            bad[k] = (l1, linf, flips[k])
    assert not bad, f"{label} FP32 parity failed: {bad}"
    return errs, flips


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


def run_oracle(orc, prob, steps, dt=None, mlp=None, fields=None):
    o = orc.Oracle(prob, mlp)
    return o.run(prob.fields if fields is None else fields, prob.dt if dt is None else dt, steps)
