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


# FP32 form: the pass bounds come from the oracle's own response to the
# disturbances FP32 brings (fp32_response).  The f-preserving face fix picks
# one of two face states on the sign of f_face - f_centre, so rounding-level
# differences flip some of those choices and move the affected cells by far
# more than the rounding; whether a run flips none, one or a few decisions
# is a matter of chance at small sizes.
F32_FACTOR = 4.0
F32_TARGET = 1e-5          # per-field rel-L1 and rel-Linf target of the FP32 form
FLIP_THRESHOLD = 1e-5      # a cell counts as reached by a flip above this x max|ref|
# relative amplitude of the face-value noise of fp32_response: a face value
# u + s h computed in FP32 from FP32 data carries the rounding of about six
# operations (two differences, the spacing factors, the slope's limiter, the
# product and the sum), a few units of 2^-24 of |u| + |s h|
FACE_NOISE = 2.0 ** -22
# the same disturbance 2^6 times larger: certain to flip face decisions, so
# its deviations show the size and the reach of the flips the method makes
# on the workload (a flip swaps one face state for the other whatever caused
# it, so their size does not depend on the amplitude)
FLIP_NOISE = 2.0 ** -16
# faces that a face treatment sets to f = 1 exactly (the simple clip) are at
# f = 1 within 2^-24 in FP32, where the signal speeds move by about
# sqrt(2 x 2^-24) = 3.5e-4 of c_hat; through the HLL dissipation a step moves
# the neighbouring cells by a fraction dt c_hat / h (<= 0.4) of that, which
# neither response reproduces (the oracle clips in FP64): rel-Linf allowance
F32_F1_LINF = 1e-4


def _oracle_fp32(orc, prob, steps, dt, rk2, mlp, fields, explicit, amp):
    o = orc.Oracle(prob, mlp)
    o.P.face_noise = amp
    mg = getattr(prob, "groups", None) is not None and len(prob.groups["kP"]) > 1
    st = {k: np.array(v, dtype=np.float64) for k, v in (prob.fields if fields is None else fields).items()}

    def rnd(s):
        for k in RAD:
            s[k] = s[k].astype(np.float32).astype(np.float64)

    rnd(st)
    if explicit:
        o.P.noise_seed = 1
        out, _ = o.explicit(st, dt)
        rnd(out)
        return out
    for step in range(steps):
        o.P.noise_seed = 16 * (step + 1)
        st, _ = (o.run_mg if mg else o.run)(st, dt, 1, rk2=rk2)
        rnd(st)
    return st


def fp32_response(orc, prob, steps, dt=None, rk2=False, mlp=None, fields=None, explicit=False):
    """The FP64 oracle disturbed where the FP32 form rounds: E and F (every
    group) rounded to FP32 at the start and after every step (storage), and
    every reconstructed face value perturbed by FACE_NOISE x (|u| + |s h|)
    times a seeded uniform number in [-1, 1) (the FP32 arithmetic of the
    face values, on whose comparison the f-preserving fix decides); the
    rest of the arithmetic in FP64.  Also the same with FLIP_NOISE.  Returns
    {"fp32": state, "flip": state} (explicit=True: the transported states of
    one explicit step)."""
    dt = prob.dt if dt is None else dt
    return {"fp32": _oracle_fp32(orc, prob, steps, dt, rk2, mlp, fields, explicit, FACE_NOISE),
            "flip": _oracle_fp32(orc, prob, steps, dt, rk2, mlp, fields, explicit, FLIP_NOISE)}


def _field_stats(a, ref, fields):
    out = {}
    for k in fields:
        d = np.abs(a[k] - ref[k])
        s1, sm = np.abs(ref[k]).sum(), np.abs(ref[k]).max()
        flips = d > FLIP_THRESHOLD * sm
        outside = d[~flips].max() if (~flips).any() else 0.0
        out[k] = dict(l1=d.sum() / s1 if s1 > 0 else d.sum(), linf=d.max() / sm if sm > 0 else d.max(),
                      flips=int(flips.sum()), linf_out=outside / sm if sm > 0 else outside)
    return out


def f32_bounds(small, big, scale=1.0, f1=False):
    """Bounds of one field from the oracle's responses (field statistics of
    the FACE_NOISE and FLIP_NOISE runs); f1: faces clipped to f = 1."""
    return dict(l1=max(F32_TARGET, F32_FACTOR * small["l1"]) * scale,
                linf=max(F32_TARGET, F32_FACTOR * small["linf"], big["linf"], F32_F1_LINF if f1 else 0.0) * scale,
                flips=max(F32_FACTOR * small["flips"] + 4, big["flips"]))


def assert_close_f32(got, ref, response, fields=ALL, label="", gas_scale=1.0, f1=False):
    """FP32 form vs the FP64 oracle, per field:
      rel-L1 <= max(1e-5 target, 4 x the oracle's rel-L1 under FP32
               disturbance (`response`["fp32"], see fp32_response));
      rel-Linf <= max(1e-5, 4 x its rel-Linf, the rel-Linf of the oracle
               under the flip-certain disturbance (`response`["flip"]));
      cells a face-fix flip has reached (deviation above 1e-5 max|ref|)
               <= max(4 x the first response's count + 4, the second's).
    Gas fields are scaled by gas_scale where c >> c_hat (E_g takes (c/c_hat)
    times the FP32 rounding of each exchange, which neither response
    reproduces); f1=True adds the rel-Linf allowance F32_F1_LINF of faces
    clipped to f = 1.  Reports rel-L1 / rel-Linf / flip cells / rel-Linf outside
    the flip cells for each field, and both responses."""
    got_s = _field_stats(got, ref, fields)
    small = _field_stats(response["fp32"], ref, fields)
    big = _field_stats(response["flip"], ref, fields)
    say(f"  {label} " + " ".join(f"{k}:{v['l1']:.1e}/{v['linf']:.1e}/{v['flips']}/{v['linf_out']:.1e}"
                                 for k, v in got_s.items()))
    for name, st in (("fp32", small), ("flip", big)):
        say(f"  {label} oracle {name} response " +
            " ".join(f"{k}:{v['l1']:.1e}/{v['linf']:.1e}/{v['flips']}" for k, v in st.items()))
    bad = {}
    for k in fields:
        scale = gas_scale if k in ("mx", "my", "mz", "Eg") else 1.0
        g, bd = got_s[k], f32_bounds(small[k], big[k], scale, f1)
        if g["l1"] > bd["l1"] or g["linf"] > bd["linf"] or (scale == 1.0 and g["flips"] > bd["flips"]):
            bad[k] = (g, bd)
    assert not bad, f"{label} FP32 parity failed: {bad}"
    return got_s, small, big


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
