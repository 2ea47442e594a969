"""GPU parity of the reflective and fixed boundaries, the irradiation heating
and the absorption-only coupling against the oracle, in both forms, and the
shadow test of Sect. 3.3 at the paper's resolution."""
import numpy as np
import pytest

from paper_2606_26268_amd import inputs as I
from tests.gpu_common import TOL_P64, assert_close, assert_close_f32, fp32_response, rel_errors, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu


def _random_problem(geometry, n, ndim, bc, seed, faces=None, kP=0.8, kR=0.5, bc_state=None):
    if faces is None:
        faces = [I.uniform_faces(n[d], 0.0, 1.0) if n[d] > 1 else np.array([0.0, 1.0]) for d in range(3)]
    p = I.make_random_state(geometry, n, ndim, seed, faces, I.PERIODIC, fmax=0.8, c_hat=3.0,
                            opacity=dict(kind=I.OPAC_CONSTANT, kP=kP, kR=kR, sigma=0.2))
    p.bc = bc
    p.bc_state = bc_state
    p.dt = 0.3 / (3.0 * sum(1.0 / (faces[d][1] - faces[d][0]) for d in range(ndim)))
    return p


BEAM = (2.0, 1.6, 0.3, -0.2)
CASES = {
    # 1D Cartesian, mirror walls at both ends
    "1d_reflect": (I.CARTESIAN, (48, 1, 1), 1,
                   [[I.REFLECT, I.REFLECT], [0, 0], [0, 0]], None),
    # 2D Cartesian: injected state on the left, wall at y = 0 (ragged tiles)
    "2d_fixed_reflect": (I.CARTESIAN, (40, 20, 1), 2,
                         [[I.FIXED, I.OUTFLOW], [I.REFLECT, I.OUTFLOW], [0, 0]],
                         [[BEAM, None], [None, None], [None, None]]),
    # 3D tiled kernel: every kind of side, ragged in x and y, reflective in z
    "3d_mixed": (I.CARTESIAN, (40, 12, 10), 3,
                 [[I.REFLECT, I.OUTFLOW], [I.FIXED, I.REFLECT], [I.REFLECT, I.REFLECT]],
                 [[None, None], [BEAM, None], [None, None]]),
    # 3D with a fixed side in z (register window ghosts)
    "3d_fixed_z": (I.CARTESIAN, (33, 9, 12), 3,
                   [[0, 0], [I.OUTFLOW, I.OUTFLOW], [I.FIXED, I.FIXED]],
                   [[None, None], [None, None], [BEAM, (1.0, -0.2, 0.1, -0.6)]]),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_boundary_parity(orc, name, precision):
    geom, n, ndim, bc, bs = CASES[name]
    p = _random_problem(geom, n, ndim, bc, seed=31, bc_state=bs)
    say(f"case {name} {precision} n={n} bc={bc}")
    ref, _ = run_oracle(orc, p, 12)
    got, _ = run_gpu(p, precision, 12)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label=name)
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 12), label=name)


def test_spherical_reflective_equator(orc):
    """Spherical (r, theta) with a mirror wall at theta = pi / 2."""
    n = (24, 16, 1)
    faces = [np.linspace(1.0, 3.0, 25), np.linspace(0.0, np.pi / 2, 17), np.array([0.0, 2 * np.pi])]
    p = _random_problem(I.SPHERICAL, n, 2, [[I.OUTFLOW, I.OUTFLOW], [I.OUTFLOW, I.REFLECT], [0, 0]], 33,
                        faces=faces)
    p.dt = 0.3 / (3.0 * (1 / (2 / 24) + 1 / (np.pi / 32)))
    say("case spherical equator wall")
    ref, _ = run_oracle(orc, p, 10)
    got, _ = run_gpu(p, "p64", 10)
    assert_close(got, ref, TOL_P64, label="sph-reflect")


@pytest.mark.parametrize("precision", ["p64", "f32"])
@pytest.mark.parametrize("absorb", [0, 1])
def test_irradiation_and_absorption_parity(orc, precision, absorb):
    n = (36, 10, 9)
    p = _random_problem(I.CARTESIAN, n, 3, [[0, 0]] * 3, seed=41, kP=5.0, kR=2.0)
    p.c = 30.0
    rng = np.random.default_rng(3)
    p.irr = np.exp(rng.standard_normal(p.fields["E"].shape)) * 2.0
    p.absorb_only = absorb
    say(f"case irradiation absorb={absorb} {precision}")
    ref, _ = run_oracle(orc, p, 8)
    got, _ = run_gpu(p, precision, 8)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label=f"irr/abs{absorb}")
    else:
        # c / c_hat = 10 amplifies the FP32 rounding of E in E_g
        assert_close_f32(got, ref, fp32_response(orc, p, 8), label=f"irr/abs{absorb}", gas_scale=10.0)


def _sensitivity(orc, p, steps, eps, ref, fields):
    """Relative change of the oracle's own result when (E, F) are perturbed
    by eps (relative, seeded noise): the conditioning of the problem."""
    rng = np.random.default_rng(0)
    f2 = {k: v.copy() for k, v in p.fields.items()}
    for k in ("E", "Fx", "Fy", "Fz"):
        f2[k] = f2[k] * (1 + eps * rng.standard_normal(f2[k].shape))
    pert, _ = run_oracle(orc, p, steps, fields=f2)
    return rel_errors(pert, ref, fields)


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_shadow_parity(orc, precision):
    """The shadow test at 140 x 40 (Sect. 3.3), absorption only, 300 steps.

    The beam is free-streaming (f = 1), where the signal speeds depend on
    sqrt(1 - f): a rounding-level change of the state moves the result by
    far more than the rounding (the oracle itself moves by 1e-7 in E and
    2e-4 in the small F_y under a 1e-15 input perturbation).  The GPU must
    agree with the oracle to within 4x that measured conditioning at the
    rounding level of its precision (and never worse than the standard
    tolerances would allow where the problem is well conditioned)."""
    p = I.make_shadow(absorb_only=1)
    steps = 300
    say(f"case shadow 140x40 {precision}")
    fields = ("E", "Fx", "Fy", "Eg")
    ref, _ = run_oracle(orc, p, steps)
    got, _ = run_gpu(p, precision, steps)
    errs = rel_errors(got, ref, fields)
    if precision == "p64":
        sens = _sensitivity(orc, p, steps, 1e-15, ref, fields)
        say("  shadow gpu/oracle vs oracle sensitivity: " +
            " ".join(f"{k}:{errs[k][0]:.1e}/{errs[k][1]:.1e} ({sens[k][0]:.1e}/{sens[k][1]:.1e})" for k in fields))
        for k in fields:
            assert errs[k][0] <= max(TOL_P64["l1"], 4 * sens[k][0]), (k, errs[k], sens[k])
            assert errs[k][1] <= max(TOL_P64["linf"], 4 * sens[k][1]), (k, errs[k], sens[k])
        return
    # FP32: E and E_g per field; the flux as one vector field (F_y is only
    # ~2e-4 of F_x here, made at the beam edges, so its own relative error
    # says little), each within the bounds the oracle's responses to the
    # FP32 disturbances give (rel-L1 and rel-Linf, as assert_close_f32)
    resp = fp32_response(orc, p, steps)

    def vec(a):
        dF = np.sqrt(sum((a[k] - ref[k]) ** 2 for k in ("Fx", "Fy", "Fz")))
        Fn = np.sqrt(sum(ref[k] ** 2 for k in ("Fx", "Fy", "Fz")))
        return dF.sum() / Fn.sum(), dF.max() / Fn.max()

    got_e = {"E": errs["E"], "Eg": errs["Eg"], "F": vec(got)}
    res = {}
    for name in ("fp32", "flip"):
        r = rel_errors(resp[name], ref, fields)
        res[name] = {"E": r["E"], "Eg": r["Eg"], "F": vec(resp[name])}
    say("  shadow f32 (oracle fp32 / flip responses): " +
        " ".join(f"{k}:{v[0]:.1e}/{v[1]:.1e} ({res['fp32'][k][0]:.1e}/{res['fp32'][k][1]:.1e}, "
                 f"{res['flip'][k][0]:.1e}/{res['flip'][k][1]:.1e})" for k, v in got_e.items()))
    for k, (l1, linf) in got_e.items():
        small, big = res["fp32"][k], res["flip"][k]
        assert l1 <= max(1e-5, 4 * small[0]), (k, l1, small)
        assert linf <= max(1e-5, 4 * small[1], big[1]), (k, linf, small, big)


def test_boundary_errors():
    from paper_2606_26268_amd import m1
    p = _random_problem(I.CARTESIAN, (16, 1, 1), 1, [[I.FIXED, I.OUTFLOW], [0, 0], [0, 0]], seed=1)
    s = m1.Solver(p, "p64")
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_explicit(s.ctx, p.dt)
    assert e.value.status == m1.M1_ESTATE
    with pytest.raises(m1.M1Error) as e:
        m1.m1_set_boundary_state(s.ctx, 0, 1, (1.0, 0.0, 0.0, 0.0))   # outflow side
    assert e.value.status == m1.M1_EINVAL
    with pytest.raises(m1.M1Error) as e:
        m1.m1_set_boundary_state(s.ctx, 0, 0, (1.0, 2.0, 0.0, 0.0))   # |F| > E
    assert e.value.status == m1.M1_EINVAL
    m1.m1_set_boundary_state(s.ctx, 0, 0, (1.0, 0.5, 0.0, 0.0))
    m1.m1_step_explicit(s.ctx, p.dt)
    m1.m1_step_implicit(s.ctx, p.dt)
    s.sync()
    s.close()
    q = _random_problem(I.CARTESIAN, (1, 1, 1), 1, [[I.REFLECT, I.REFLECT], [0, 0], [0, 0]], seed=2)
    with pytest.raises(m1.M1Error) as e:
        m1.Solver(q, "p64")
    assert e.value.status == m1.M1_EINVAL
