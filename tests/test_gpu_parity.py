"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Small cases span several 256-thread tiles with ragged tails and every
geometry / boundary / opacity kind; full-size cases use the benchmark
workloads (128^3 for 50 steps, 256^3 and the 192x96x192 spherical grid for
a few steps each).
"""
import numpy as np
import pytest

from paper_2606_26268_amd import inputs as I
from tests.gpu_common import (ALL, RAD, TOL_P64, TOL_P64_F1, assert_close, assert_close_f32, fp32_response, rel_errors,
                               run_gpu, run_oracle, say)

pytestmark = pytest.mark.gpu


def _faces(geom, n, ndim):
    if geom == I.CARTESIAN:
        return [I.uniform_faces(n[d], 0.0, 1.0) if d < ndim else np.array([0.0, 1.0]) for d in range(3)]
    if geom == I.CYLINDRICAL:
        return [I.uniform_faces(n[0], 0.5, 2.0), I.uniform_faces(n[1], 0.0, 2 * np.pi),
                I.uniform_faces(n[2], -1.0, 1.0)]
    return [np.geomspace(1.0, 10.0, n[0] + 1), I.uniform_faces(n[1], 0.0, np.pi),
            I.uniform_faces(n[2], 0.0, 2 * np.pi)]


def _bc(geom):
    if geom == I.CARTESIAN:
        return [[I.PERIODIC] * 2, [I.OUTFLOW] * 2, [I.PERIODIC] * 2]
    if geom == I.CYLINDRICAL:
        return [[I.OUTFLOW] * 2, [I.PERIODIC] * 2, [I.OUTFLOW] * 2]
    return [[I.OUTFLOW] * 2, [I.OUTFLOW] * 2, [I.PERIODIC] * 2]


CASES = [
    (I.CARTESIAN, (301, 1, 1), 1), (I.CARTESIAN, (37, 23, 1), 2), (I.CARTESIAN, (37, 23, 19), 3),
    (I.CYLINDRICAL, (45, 1, 1), 1), (I.CYLINDRICAL, (29, 17, 1), 2), (I.CYLINDRICAL, (21, 13, 11), 3),
    (I.SPHERICAL, (50, 1, 1), 1), (I.SPHERICAL, (27, 14, 1), 2), (I.SPHERICAL, (24, 12, 22), 3),
]


def _problem(geom, n, ndim, seed, opacity=None, vmax=0.3):
    p = I.make_random_state(geom, n, ndim, seed, _faces(geom, n, ndim), _bc(geom), fmax=0.9,
                            c_hat=3.0, opacity=opacity, vmax=vmax)
    return p


@pytest.mark.parametrize("geom,n,ndim", CASES)
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_small_grids_all_geometries(orc, geom, n, ndim, precision):
    say(f"case geom={geom} n={n} ndim={ndim} {precision}")
    p = _problem(geom, n, ndim, seed=100 + 10 * geom + ndim)
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    steps = 10
    ref, cnt = o.run(p.fields, dt, steps)
    got, diag = run_gpu(p, precision, steps, dt=dt)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, steps, dt=dt), label="f32")
    assert diag["counters"][:3] == list(cnt[:3])


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_transport_only_matches_oracle(orc, precision):
    """One explicit step (E*, F*) on a 3D spherical random state."""
    from paper_2606_26268_amd import m1
    p = _problem(I.SPHERICAL, (24, 12, 22), 3, seed=7)
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, _ = o.explicit(p.fields, dt)
    s = m1.Solver(p, precision=precision)
    m1.m1_step_explicit(s.ctx, dt)
    got = s.transported()
    s.close()
    if precision == "p64":
        assert_close(got, ref, TOL_P64, fields=RAD, label="transport")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 1, dt=dt, explicit=True), fields=RAD, label="transport")


@pytest.mark.parametrize("kind", ["powerlaw", "table"])
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_temperature_dependent_opacities(orc, kind, precision):
    if kind == "powerlaw":
        op = dict(kind=I.OPAC_POWERLAW, k0=2.0, rho0=1.0, alpha=1.0, T0=1.0, beta=-3.5, sigma=0.3)
    else:
        op = I.make_table()
        op["lr_off"], op["lt_off"] = -5.0, 4.0
    p = _problem(I.CARTESIAN, (33, 17, 9), 3, seed=21, opacity=op)
    if kind == "table":
        p.c = 5.0 * p.c_hat
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, _ = o.run(p.fields, dt, 10)
    got, _ = run_gpu(p, precision, 10, dt=dt)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label=kind)
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 10, dt=dt), label=kind)


def test_stiff_reduced_speed_of_light(orc):
    """c / c_hat = 1e4 and large absorption: the FP64 implicit solve keeps parity."""
    op = dict(kind=I.OPAC_CONSTANT, kP=30.0, kR=10.0, sigma=0.0)
    p = _problem(I.CARTESIAN, (40, 20, 1), 2, seed=5, opacity=op)
    p.c = 1e4 * p.c_hat
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, cnt = o.run(p.fields, dt, 20)
    assert cnt[3] == 0
    got, _ = run_gpu(p, "p64", 20, dt=dt)
    assert_close(got, ref, TOL_P64, label="stiff p64")
    # FP32 storage of E: the gas energy receives (c/c_hat) x the FP32 rounding
    # of each exchange, a random walk of size (c/c_hat) eps32 sqrt(steps) E/E_g
    f = p.fields
    gas_scale = max(1.0, p.c / p.c_hat * 2.0 ** -24 * np.sqrt(20) * f["E"].max() / np.abs(f["Eg"]).mean() / 1e-5 * 4)
    got, _ = run_gpu(p, "f32", 20, dt=dt)
    assert_close_f32(got, ref, fp32_response(orc, p, 20, dt=dt), label="stiff f32", gas_scale=gas_scale)


def test_c0_full_run(orc):
    p = I.make_c0()
    ref, cnt = run_oracle(orc, p, p.steps)
    got, diag = run_gpu(p, "p64", p.steps)
    assert_close(got, ref, TOL_P64, label="c0 p64")
    assert diag["counters"] == [0, 0, 0, 0] and (cnt == 0).all()


@pytest.fixture(scope="module")
def c1_ref(orc):
    p = I.make_c1()
    say("oracle c1 (128^3, 50 steps)")
    ref, cnt = run_oracle(orc, p, p.steps)
    return p, ref, cnt


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_c1_full_run(orc, c1_ref, precision):
    p, ref, cnt = c1_ref
    got, diag = run_gpu(p, precision, p.steps)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="c1 p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, p.steps), label="c1 f32")
    assert diag["counters"][:3] == [0, 0, 0]


def test_c2_full_size_steps(orc):
    """256^3: two full steps against the oracle in both forms."""
    p = I.make_c2()
    say("oracle c2 (256^3, 2 steps)")
    ref, _ = run_oracle(orc, p, 2)
    got, _ = run_gpu(p, "p64", 2)
    assert_close(got, ref, TOL_P64, label="c2 p64")
    got, _ = run_gpu(p, "f32", 2)
    assert_close_f32(got, ref, fp32_response(orc, p, 2), label="c2 f32")


def test_c3_full_size_steps(orc):
    """Spherical 192x96x192 with the bilinear table: three full steps."""
    p = I.make_c3()
    say("oracle c3 (192x96x192, 3 steps)")
    ref, _ = run_oracle(orc, p, 3)
    got, _ = run_gpu(p, "p64", 3)
    assert_close(got, ref, TOL_P64, label="c3 p64")
    got, _ = run_gpu(p, "f32", 3)
    assert_close_f32(got, ref, fp32_response(orc, p, 3), label="c3 f32")


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_c3_reduced_100_steps(orc, precision):
    p = I.make_c3(nr=48, nth=24, nph=48, dt=4.0e-5)
    ref, _ = run_oracle(orc, p, 100)
    got, diag = run_gpu(p, precision, 100)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="c3 reduced p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 100), label="c3 reduced f32")


def test_determinism_and_conservation():
    p = I.make_random_state(I.CARTESIAN, (40, 30, 20), 3, 9, _faces(I.CARTESIAN, (40, 30, 20), 3),
                            [[I.PERIODIC] * 2] * 3, fmax=0.7, c_hat=2.0,
                            opacity=dict(kind=I.OPAC_CONSTANT, kP=2.0, kR=1.0, sigma=0.5))
    p.c = 7.0 * p.c_hat
    from paper_2606_26268_amd import m1
    s = m1.Solver(p, "p64")
    d0 = s.diagnostics()
    dt = s.max_dt(0.4)
    s.step(dt, 50)
    a = s.state()
    d1 = s.diagnostics()
    s.close()
    b, _ = run_gpu(p, "p64", 50, dt=dt)
    for k in ALL:
        assert np.array_equal(a[k], b[k]), k
    assert abs(d1["total_energy"] - d0["total_energy"]) <= 1e-13 * abs(d0["total_energy"])
    for q in range(3):
        assert abs(d1["momentum"][q] - d0["momentum"][q]) <= 1e-13 * (abs(d0["momentum"][q]) + d0["rad_energy"])


def test_error_paths():
    from paper_2606_26268_amd import m1
    p = _problem(I.CARTESIAN, (16, 8, 4), 3, seed=3)
    s = m1.Solver(p, "p64")
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_implicit(s.ctx, 1e-3)
    assert e.value.status == m1.M1_ESTATE
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_explicit(s.ctx, -1.0)
    assert e.value.status == m1.M1_EINVAL
    bad = dict(s.t)
    import torch
    raw = torch.zeros(p.ncells + 1, dtype=torch.float64, device="cuda")
    bad["E"] = raw[1:]
    with pytest.raises(m1.M1Error) as e:
        m1.m1_bind_state(s.ctx, bad)
    assert e.value.status == m1.M1_EINVAL
    s.close()


def test_free_streaming_beam_2d(orc):
    """The Sect. 3.2 oblique beam (f = 1 inside the beam, E ratio 1e8) on a
    reduced 100x100 grid, 60 steps, FP64.  Near f = 1 the signal speeds are
    square-root sensitive to rounding of f, so the tolerance is looser."""
    p = I.make_beam(N=100, steps=60)
    ref, cnt = run_oracle(orc, p, p.steps)
    got, diag = run_gpu(p, "p64", p.steps)
    assert_close(got, ref, TOL_P64_F1, fields=RAD, label="beam p64")
    assert diag["counters"][:3] == list(cnt[:3])


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_rk2_steps(orc, precision):
    """m1_step_rk2 vs the oracle's RK2 on a spherical grid with the table."""
    op = I.make_table()
    p = _problem(I.SPHERICAL, (24, 12, 22), 3, seed=41, opacity=op)
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, cnt = o.run(p.fields, dt, 8, rk2=True)
    from paper_2606_26268_amd import m1
    s = m1.Solver(p, precision, second_order=True)
    s.step(dt, 8, rk2=True)
    got = s.state()
    s.close()
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="rk2 p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 8, dt=dt, rk2=True), label="rk2 f32")


def test_rk2_needs_second_order():
    """Without m1_params.second_order the context holds no buffer for the
    second-order step, and the step is refused instead of allocating."""
    from paper_2606_26268_amd import m1
    p = _problem(I.CARTESIAN, (16, 8, 4), 3, seed=3)
    s = m1.Solver(p, "p64")
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_rk2(s.ctx, 1e-3)
    assert e.value.status == m1.M1_ESTATE
    s.close()


@pytest.mark.parametrize("recon,riemann", [(1, 0), (2, 0), (0, 1)])
def test_face_treatment_and_riemann_variants(orc, recon, riemann):
    """PLUTO / clip face treatments and the Lax-Friedrichs flux, 3D and 2D."""
    for geom, n, ndim in ((I.CARTESIAN, (33, 17, 9), 3), (I.SPHERICAL, (27, 14, 1), 2)):
        p = _problem(geom, n, ndim, seed=51 + recon + 3 * riemann)
        p.recon, p.riemann = recon, riemann
        o = orc.Oracle(p)
        dt = o.max_dt(0.4)
        ref, cnt = o.run(p.fields, dt, 6)
        got, diag = run_gpu(p, "p64", 6, dt=dt)
        # the clip sets faces to f = 1 exactly, where the speeds are sqrt-sensitive
        tol = TOL_P64_F1 if recon == 2 else TOL_P64
        assert_close(got, ref, tol, label=f"recon {recon} riemann {riemann} ndim {ndim}")
        assert diag["counters"][:3] == list(cnt[:3])


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_flux_below_the_normal_range(orc, precision):
    """Radiation fluxes whose squared norm underflows to subnormal numbers
    (the numerical tail ahead of a front after many steps): |F| of 1e-20 to
    1e-22 in FP32, 1e-155 to 1e-161 in FP64, on a uniform E = 1.  Their
    inverse squares overflow; the closure and the geometric sources must take
    such a flux as directionless and stay finite.  One transport step against
    the oracle (Cartesian: every radiation field, relative to its own scale;
    spherical: E, and F against the scale E of the rounding of the
    well-balanced isotropic pressure, which outgrows the tiny flux at once),
    then four full steps, which must stay finite.  Before the fix the FP64
    form returned NaN fluxes here."""
    from paper_2606_26268_amd import m1
    lo, hi = (-22.0, -20.0) if precision == "f32" else (-161.0, -155.0)
    for geom, n in ((I.CARTESIAN, (37, 23, 19)), (I.SPHERICAL, (24, 12, 22))):
        say(f"case subnormal |F|^2 geom={geom} n={n} {precision}")
        p = I.make_uniform(geom, n, 3, faces=_faces(geom, n, 3), kP=1.0, kR=2.0, sigma=0.5)
        p.bc = _bc(geom)
        rng = np.random.default_rng(41)
        for k in ("Fx", "Fy", "Fz"):
            p.fields[k] = rng.choice([-1.0, 1.0], p.shape) * 10.0 ** rng.uniform(lo, hi, p.shape)
            if precision == "f32":
                p.fields[k] = p.fields[k].astype(np.float32).astype(np.float64)
        o = orc.Oracle(p)
        dt = o.max_dt(0.4)
        ref, _ = o.explicit(p.fields, dt)
        s = m1.Solver(p, precision=precision)
        m1.m1_step_explicit(s.ctx, dt)
        got = s.transported()
        s.close()
        for k in RAD:
            assert np.isfinite(got[k]).all(), k
        close = assert_close if precision == "p64" else assert_close_f32
        args = (TOL_P64,) if precision == "p64" else (fp32_response(orc, p, 1, dt=dt, explicit=True),)
        if geom == I.CARTESIAN and precision == "f32":
            # |F|^2 of 1e-40 to 1e-44 keeps only a few significant bits in
            # FP32, so some f-preserving face decisions (|F_face| against
            # |F_centre|) flip; the transverse flux components diffuse through
            # those face values
            close(got, ref, *args, fields=("E",), label="subnormal transport")
            for k, (l1, linf) in rel_errors(got, ref, ("Fx", "Fy", "Fz")).items():
                assert l1 <= 1e-4 and linf <= 1e-2, (k, l1, linf)
        elif geom == I.CARTESIAN:
            close(got, ref, *args, fields=RAD, label="subnormal transport")
        else:
            close(got, ref, *args, fields=("E",), label="subnormal transport")
            tol = 1e-12 if precision == "p64" else 1e-5
            for k in ("Fx", "Fy", "Fz"):
                assert np.abs(got[k] - ref[k]).max() <= tol * ref["E"].max(), k
        full, _ = run_gpu(p, precision, 4, dt=dt)
        for k in ALL:
            assert np.isfinite(full[k]).all(), k


THIN = [
    (I.CARTESIAN, (40, 9, 1)), (I.CARTESIAN, (5, 3, 2)), (I.CARTESIAN, (1, 1, 1)), (I.CARTESIAN, (33, 1, 4)),
    (I.CYLINDRICAL, (20, 3, 2)), (I.SPHERICAL, (24, 12, 2)),
]


@pytest.mark.parametrize("geom,n", THIN)
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_thin_and_tiny_3d_grids(orc, geom, n, precision):
    """Three-dimensional grids with one, two or three cells along some
    directions (periodic wraps that reach the same cell twice, outflow ghosts
    that all copy one cell) and a single-cell grid, through the tiled
    transport kernel, against the oracle."""
    say(f"case thin 3D geom={geom} n={n} {precision}")
    p = _problem(geom, n, 3, seed=300 + sum(n))
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, cnt = o.run(p.fields, dt, 5)
    got, diag = run_gpu(p, precision, 5, dt=dt)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="thin p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 5, dt=dt), label="thin f32")
    assert diag["counters"][:3] == list(cnt[:3])


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_pulse_long_run(orc, precision):
    """The pulse recipe on 64^3 cells for 40 second-order steps: the front
    crosses the box's outer cells, where the flux grows from exactly zero
    through values whose squares leave the normal range (the regime in which
    the FP32 closure once returned NaN).  Radiation against the oracle; the
    gas is judged against the scales it inherits rounding from, as in the
    full-size pulse test."""
    p = I.make_pulse3d(N=64, steps=40)
    say(f"case pulse 64^3 rk2 {precision}, 40 steps")
    ref, _ = orc.Oracle(p).run(p.fields, p.dt, p.steps, rk2=True)
    from paper_2606_26268_amd import m1
    s = m1.Solver(p, precision, second_order=True)
    s.step(p.dt, p.steps, rk2=True)
    got = s.state()
    s.close()
    for k in ALL:
        assert np.isfinite(got[k]).all(), k
    if precision == "p64":
        assert_close(got, ref, TOL_P64, fields=RAD, label="pulse 64 p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, p.steps, rk2=True), fields=RAD, label="pulse 64 f32")
    tol = 1e-14 if precision == "p64" else 1e-6
    for c in ("x", "y", "z"):
        d = np.abs(got["m" + c] - ref["m" + c])
        assert d.sum() <= tol * (np.abs(ref["F" + c]).sum() / p.c_hat), c
    es = (p.c / p.c_hat) * np.abs(ref["E"]).max()
    assert np.abs(got["Eg"] - ref["Eg"]).max() <= 10 * tol * es


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_injected_unrealizable_cells_are_fixed_like_the_oracle(orc, precision):
    """Host-forced fix-ups: two cells of a 3D random state get |F| = 3 E and
    |F| = 1.5 E (f > 1, unrealizable), and the energy floor is raised to the
    0.5 % quantile of E so that the positivity floor acts in a few cells.
    After two steps the fix-up counters (energy floor, f <= 1 after transport
    and after the implicit step) equal the oracle's, the first two non-zero
    (2 and 2), and the state matches the oracle as usual."""
    p = _problem(I.CARTESIAN, (24, 16, 12), 3, seed=77)
    E = p.fields["E"]
    for idx, fac in (((3, 5, 7), 3.0), ((9, 2, 20), 1.5)):
        fn = np.sqrt(p.fields["Fx"][idx] ** 2 + p.fields["Fy"][idx] ** 2 + p.fields["Fz"][idx] ** 2)
        scale = fac * E[idx] / fn
        for k in ("Fx", "Fy", "Fz"):
            p.fields[k][idx] *= scale
    p.e_floor = float(np.quantile(E, 0.005))
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, cnt = o.run(p.fields, dt, 2)
    got, diag = run_gpu(p, precision, 2, dt=dt)
    say(f"  injected fix-ups: oracle {list(cnt[:3])}, GPU {diag['counters'][:3]}")
    assert cnt[0] > 0 and cnt[1] > 0, cnt
    if precision == "p64":
        assert diag["counters"][:3] == list(cnt[:3])
        assert_close(got, ref, TOL_P64, label="injected p64")
    else:
        # FP32 rounding can move a cell across the floor: counts within one
        assert all(abs(a - b) <= 1 for a, b in zip(diag["counters"][:3], cnt[:3])), (diag["counters"], cnt)
        assert_close_f32(got, ref, fp32_response(orc, p, 2, dt=dt), label="injected f32")


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_checkpoint_and_resume_is_bitwise(precision):
    """Checkpoint / resume: the caller owns the state, so a checkpoint is a
    copy of its arrays; a new context bound to the copy (the opacity cache
    re-derived from the gas state) continues bit for bit like the context
    that kept stepping (spherical grid, bilinear table: temperature-dependent
    opacities)."""
    from paper_2606_26268_amd import m1
    p = I.make_c3(nr=24, nth=12, nph=20, dt=4.0e-5)
    s = m1.Solver(p, precision)
    s.step(p.dt, 3)
    saved = s.state()
    s.step(p.dt, 3)
    a = s.state()
    s.close()
    q = I.Problem(**{**p.__dict__, "fields": saved})
    r = m1.Solver(q, precision)
    r.step(p.dt, 3)
    b = r.state()
    r.close()
    for k in ALL:
        assert np.array_equal(a[k], b[k]), k


def _mlp_weights():
    th = I.mlp_init(7)
    rng = np.random.default_rng(7)
    tab = I.make_table()
    a, b = tab["log10_kP"].astype(np.float64), tab["log10_kR"].astype(np.float64)
    return dict(theta=(th + 0.05 * rng.normal(size=th.size)).astype(np.float32),
                norm=np.array([a.mean(), a.std(), b.mean(), b.std()]))


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_streaming_reads_change_no_bit(precision):
    """The implicit step's two ways of reading its inputs (m1_params.
    stream_reads: nontemporal loads, or plain ones) give the same bits, for
    the table, the network, the second-order step and eight groups; the
    automatic choice takes one of them by the step's size, so both kernels
    of each form are checked here on small grids."""
    from paper_2606_26268_amd import m1
    cases = [("table", I.make_c3(nr=24, nth=12, nph=20, dt=4.0e-5), None, False),
             ("table rk2", I.make_c3(nr=24, nth=12, nph=20, dt=4.0e-5), None, True),
             ("network", I.make_c4(nr=24, nth=12, nph=20, dt=4.0e-5), _mlp_weights(), False),
             ("groups", I.make_multigroup(8, (16, 16, 16)), None, False)]
    for name, p, mlp, rk2 in cases:
        say(f"case stream_reads {name} {precision}")
        out = []
        for mode in (m1.M1_STREAM_ON, m1.M1_STREAM_OFF):
            p.stream_reads = mode
            s = m1.Solver(p, precision, mlp=mlp, second_order=rk2)
            s.step(p.dt, 3, rk2=rk2)
            out.append(s.state())
            s.close()
        for k in out[0]:
            assert np.array_equal(out[0][k], out[1][k]), (name, k)


@pytest.mark.parametrize("shape", [(128, 128), (7, 5), (2, 2)])
def test_table_lookup_matches_oracle_everywhere(orc, shape):
    """The bilinear table on the GPU (m1_opacity_eval, FP64; it reads each
    table cell's four node values from one record) against the oracle's
    lookup: random points over and well beyond the axes (both clamps), every
    node, and the midpoints of the first and last cells of every row; on the
    benchmark's 128 x 128 nodes, a small ragged table and the smallest one."""
    import torch
    from paper_2606_26268_amd import m1
    nr, nt = shape
    tab = I.make_table(nr, nt)
    p = I.make_uniform(I.CARTESIAN, (64, 1, 1), 1)
    p.opacity = tab
    s = m1.Solver(p, "p64")
    rng = np.random.default_rng(11)
    lr_axis = tab["lr0"] + (tab["lr1"] - tab["lr0"]) * np.arange(nr) / (nr - 1)
    lt_axis = tab["lt0"] + (tab["lt1"] - tab["lt0"]) * np.arange(nt) / (nt - 1)
    span_r, span_t = tab["lr1"] - tab["lr0"], tab["lt1"] - tab["lt0"]
    lr = [rng.uniform(tab["lr0"] - 0.3 * span_r, tab["lr1"] + 0.3 * span_r, 4099)]
    lt = [rng.uniform(tab["lt0"] - 0.3 * span_t, tab["lt1"] + 0.3 * span_t, 4099)]
    LT, LR = np.meshgrid(lt_axis, lr_axis, indexing="ij")
    lr.append(LR.ravel())
    lt.append(LT.ravel())
    mid_r = 0.5 * (lr_axis[[0, -2]] + lr_axis[[1, -1]])
    MT, MR = np.meshgrid(lt_axis, mid_r, indexing="ij")
    lr.append(MR.ravel())
    lt.append(MT.ravel())
    lr, lt = np.concatenate(lr), np.concatenate(lt)
    rho, T = 10 ** (lr - tab["lr_off"]), 10 ** (lt - tab["lt_off"])
    n = rho.size
    kP = torch.empty(n, dtype=torch.float64, device="cuda")
    kR = torch.empty_like(kP)
    m1.m1_opacity_eval(s.ctx, n, torch.from_numpy(rho).to("cuda"), torch.from_numpy(T).to("cuda"), kP, kR)
    s.sync()
    s.close()
    rP, rR = orc.Oracle(p).opacity(rho, T)
    eP = np.abs(kP.cpu().numpy() / rP - 1).max()
    eR = np.abs(kR.cpu().numpy() / rR - 1).max()
    say(f"  table {nr}x{nt}: {n} points, max rel diff P {eP:.1e} R {eR:.1e}")
    assert eP <= 1e-12 and eR <= 1e-12
