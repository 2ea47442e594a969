"""Pins of the oracle's boundary conditions and extra source terms:

* reflective boundaries: a run with mirror walls equals the matching half of
  a run on the doubled, mirror-symmetric periodic domain (the symmetry a
  reflective wall stands for), bit for bit on dyadic grids;
* fixed (inflow) boundaries: a beam injected at f = 1 into an empty medium
  fills it at the reduced speed of light and leaves a uniform state behind
  the front (free streaming, Sect. 3.2); a fixed state equal to the interior
  keeps a uniform field uniform;
* irradiation (Sect. 2.9): the solution satisfies the paper's linear system
  with the modified S_1 row, the deposited energy q dt appears in the total,
  the transparent limit and the relaxation limit solved independently;
* absorption only (Sect. 3.3): the continuous absorption rate, radiation
  never grows, energy conservation;
* the shadow test of Sect. 3.3 (reduced grid): a sharp shadow behind the
  opaque spheroid, the lit region attenuated by the background absorption.
"""
import math

import numpy as np
import pytest

from paper_2606_26268_amd import inputs as I

NAMES = ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")


def _random_fields(rng, shape, fmax=0.8):
    E = np.exp(0.5 * rng.standard_normal(shape))
    u = rng.uniform(0, fmax, shape)
    ct = rng.uniform(-1, 1, shape)
    ph = rng.uniform(0, 2 * np.pi, shape)
    st = np.sqrt(1 - ct ** 2)
    rho = np.exp(0.3 * rng.standard_normal(shape))
    T = np.exp(0.2 * rng.standard_normal(shape))
    return dict(E=E, Fx=u * E * st * np.cos(ph), Fy=u * E * st * np.sin(ph), Fz=u * E * ct,
                rho=rho, mx=np.zeros(shape), my=np.zeros(shape), mz=np.zeros(shape),
                Eg=rho * T / (2.0 / 3.0))


def _problem(n, ndim, faces, bc, fields, kP=0.7, kR=0.4, c_hat=1.0):
    return I.Problem("t", I.CARTESIAN, ndim, tuple(n), faces, bc, c_hat=c_hat, c=c_hat,
                     opacity=dict(kind=I.OPAC_CONSTANT, kP=kP, kR=kR, sigma=0.1), fields=fields)


def _faces(n, hi):
    return I.uniform_faces(n, 0.0, hi)


# ---------------------------------------------------------------------------
# reflective walls
# ---------------------------------------------------------------------------

def _mirror(fields, axis, normal):
    """Append the mirror image of every field along array axis `axis`,
    reversing the flux component `normal`."""
    out = {}
    for k, a in fields.items():
        m = np.flip(a, axis=axis)
        if k == normal:
            m = -m
        out[k] = np.ascontiguousarray(np.concatenate([a, m], axis=axis))
    return out


def test_reflective_walls_equal_mirrored_periodic_domain_1d(orc):
    n = 32
    rng = np.random.default_rng(11)
    f = _random_fields(rng, (1, 1, n))
    one = [np.array([0.0, 1.0])] * 2
    pa = _problem((n, 1, 1), 1, [_faces(n, 1.0)] + one, [[I.REFLECT, I.REFLECT], [0, 0], [0, 0]], f)
    pb = _problem((2 * n, 1, 1), 1, [_faces(2 * n, 2.0)] + one, [[0, 0], [0, 0], [0, 0]], _mirror(f, 2, "Fx"))
    dt = 0.4 / n
    ra, ca = orc.Oracle(pa).run(pa.fields, dt, 20)
    rb, cb = orc.Oracle(pb).run(pb.fields, dt, 20)
    for k in NAMES:
        np.testing.assert_array_equal(ra[k], rb[k][..., :n], err_msg=k)
    # and the doubled run stayed mirror-symmetric
    np.testing.assert_array_equal(rb["E"][..., :n], np.flip(rb["E"][..., n:], axis=2))


def test_reflective_walls_equal_mirrored_periodic_domain_2d(orc):
    nx, ny = 16, 16
    rng = np.random.default_rng(12)
    f = _random_fields(rng, (1, ny, nx))
    one = np.array([0.0, 1.0])
    pa = _problem((nx, ny, 1), 2, [_faces(nx, 1.0), _faces(ny, 1.0), one],
                  [[0, 0], [I.REFLECT, I.REFLECT], [0, 0]], f)
    pb = _problem((nx, 2 * ny, 1), 2, [_faces(nx, 1.0), _faces(2 * ny, 2.0), one],
                  [[0, 0], [0, 0], [0, 0]], _mirror(f, 1, "Fy"))
    dt = 0.4 / (nx + ny)
    ra, _ = orc.Oracle(pa).run(pa.fields, dt, 10)
    rb, _ = orc.Oracle(pb).run(pb.fields, dt, 10)
    for k in NAMES:
        np.testing.assert_array_equal(ra[k], rb[k][:, :ny, :], err_msg=k)


def test_reflective_wall_with_outflow_partner_matches_half_of_symmetric_run(orc):
    """A wall at y = 0 and outflow at the far side (the shadow test's
    arrangement) against the full symmetric domain with outflow on both sides."""
    nx, ny = 8, 12
    rng = np.random.default_rng(13)
    f = _random_fields(rng, (1, ny, nx))
    one = np.array([0.0, 1.0])
    pa = _problem((nx, ny, 1), 2, [_faces(nx, 1.0), _faces(ny, 1.0), one],
                  [[0, 0], [I.REFLECT, I.OUTFLOW], [0, 0]], f)
    # rows 0 .. ny-1 hold the mirror image (F_y reversed), rows ny .. 2ny-1 the
    # original: the wall sits between rows ny-1 and ny
    fb = {k: np.ascontiguousarray(np.concatenate([(-1 if k == "Fy" else 1) * np.flip(v, axis=1), v], axis=1))
          for k, v in f.items()}
    faces_b = I.uniform_faces(2 * ny, -1.0, 1.0)
    pb = _problem((nx, 2 * ny, 1), 2, [_faces(nx, 1.0), faces_b, one], [[0, 0], [I.OUTFLOW, I.OUTFLOW], [0, 0]], fb)
    dt = 0.4 / (nx + ny)
    ra, _ = orc.Oracle(pa).run(pa.fields, dt, 6)
    rb, _ = orc.Oracle(pb).run(pb.fields, dt, 6)
    # the face coordinates of the two grids round differently: agreement to
    # rounding, not bit for bit
    for k in NAMES:
        np.testing.assert_allclose(ra[k], rb[k][:, ny:, :], rtol=1e-13, atol=1e-13 * np.abs(ra[k]).max(), err_msg=k)


# ---------------------------------------------------------------------------
# fixed (inflow) boundaries
# ---------------------------------------------------------------------------

def test_fixed_boundary_injects_a_free_streaming_beam(orc):
    n = 200
    one = [np.array([0.0, 1.0])] * 2
    f = {k: np.zeros((1, 1, n)) for k in NAMES}
    f["E"][:] = 1e-8
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.5
    p = I.Problem("beam1d", I.CARTESIAN, 1, (n, 1, 1), [_faces(n, 1.0)] + one,
                  [[I.FIXED, I.OUTFLOW], [0, 0], [0, 0]], c_hat=1.0, c=1.0,
                  opacity=dict(kind=I.OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.0), fields=f,
                  bc_state=[[(1.0, 1.0, 0.0, 0.0), None], [None, None], [None, None]])
    dt = 0.4 / n
    steps = 250                                   # t = 0.5
    r, cnt = orc.Oracle(p).run(f, dt, steps)
    x = (np.arange(n) + 0.5) / n
    E = r["E"][0, 0]
    t = steps * dt
    # front where E crosses one half: at c_hat t within a few cells
    front = x[np.argmax(E < 0.5)]
    assert abs(front - t) < 4.0 / n, front
    behind = x < t - 10.0 / n
    assert np.allclose(E[behind], 1.0, rtol=1e-6)
    assert np.allclose(r["Fx"][0, 0][behind], 1.0, rtol=1e-6)
    assert np.all(E[x > t + 10.0 / n] < 1e-6)


def test_fixed_state_equal_to_interior_keeps_uniform_field(orc):
    n = 24
    one = [np.array([0.0, 1.0])] * 2
    U = (2.0, 0.3, -0.2, 0.1)
    f = {k: np.zeros((1, 1, n)) for k in NAMES}
    f["E"][:], f["Fx"][:], f["Fy"][:], f["Fz"][:] = U
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.5
    p = I.Problem("u", I.CARTESIAN, 1, (n, 1, 1), [_faces(n, 1.0)] + one,
                  [[I.FIXED, I.FIXED], [0, 0], [0, 0]], c_hat=1.0, c=1.0,
                  opacity=dict(kind=I.OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.0), fields=f,
                  bc_state=[[U, U], [None, None], [None, None]])
    r, _ = orc.Oracle(p).run(f, 0.01, 30)
    for k, v in zip(("E", "Fx", "Fy", "Fz"), U):
        np.testing.assert_allclose(r[k], v, rtol=1e-14, atol=1e-15)


# ---------------------------------------------------------------------------
# irradiation
# ---------------------------------------------------------------------------

def test_irradiated_cell_solves_the_modified_system(orc):
    rng = np.random.default_rng(5)
    for _ in range(300):
        Es = math.exp(rng.normal())
        rho = math.exp(rng.normal())
        Cv = rho * 1.5
        T = math.exp(0.3 * rng.normal())
        kP = math.exp(2 * rng.normal())
        dt = 10 ** rng.uniform(-5, -1)
        c_hat = 10 ** rng.uniform(0, 2)
        c = c_hat * 10 ** rng.uniform(0, 3)
        S = Cv * T * 10 ** rng.uniform(-4, 0)
        E1, T1, E1c, T1c = orc.implicit_cell(Es, Cv, T, kP, rho, dt, c_hat, c, 1.0, S)
        gr, g = dt * c_hat * kP * rho, dt * c * kP * rho
        aT3, aT4 = T ** 3, T ** 4
        # the two rows of the implicit matrix, S_1 carrying the deposited energy
        r1 = (1 + gr) * E1 - 4 * gr * aT3 * T1 - (Es - 3 * gr * aT4)
        r2 = -g * E1 + (Cv + 4 * g * aT3) * T1 - (Cv * T + 3 * g * aT4 + S)
        s1 = (1 + gr) * E1 + 4 * gr * aT3 * T1 + Es + 3 * gr * aT4
        s2 = g * E1 + (Cv + 4 * g * aT3) * T1 + Cv * T + 3 * g * aT4 + S
        assert abs(r1) <= 1e-14 * s1 and abs(r2) <= 1e-14 * s2
        assert abs(E1 - E1c) <= 1e-9 * (E1 + gr * aT4)


def test_irradiation_transparent_and_relaxation_limits(orc):
    Es, Cv, T, rho, c_hat, c, S = 0.7, 3.0, 1.2, 2.0, 5.0, 50.0, 0.4
    # kappa = 0: radiation untouched, the gas takes all of S
    E1, T1, _, _ = orc.implicit_cell(Es, Cv, T, 0.0, rho, 0.1, c_hat, c, 1.0, S)
    assert abs(E1 - Es) <= 2e-16 * Es and abs(T1 - (T + S / Cv)) <= 1e-15 * T
    # kappa -> infinity: the linearised equilibrium E' = a (4 T^3 T' - 3 T^4)
    # with the total C_v T' + (c/c_hat) E' = C_v T + (c/c_hat) E* + S
    E1, T1, _, _ = orc.implicit_cell(Es, Cv, T, 1e12, rho, 0.1, c_hat, c, 1.0, S)
    r = c / c_hat
    T_lim = (Cv * T + r * Es + S + 3 * r * T ** 4) / (Cv + 4 * r * T ** 3)
    E_lim = 4 * T ** 3 * T_lim - 3 * T ** 4
    assert abs(T1 - T_lim) <= 1e-9 * T_lim and abs(E1 - E_lim) <= 1e-9 * E_lim


def test_irradiation_deposits_q_dt_in_the_total(orc):
    n = (6, 5, 4)
    rng = np.random.default_rng(7)
    f = _random_fields(rng, (n[2], n[1], n[0]))
    q = np.exp(rng.standard_normal(f["E"].shape))
    faces = [_faces(m, 1.0) for m in n]
    p = _problem(n, 3, faces, [[0, 0]] * 3, f, kP=3.0, kR=2.0, c_hat=2.0)
    p.c = 20.0
    p.irr = q
    o = orc.Oracle(p)
    dt = 0.01
    star = {k: f[k] for k in ("E", "Fx", "Fy", "Fz")}
    out, _ = o.implicit(f, star, dt)
    r = p.c / p.c_hat
    before = f["Eg"] + r * f["E"] + q * dt
    after = out["Eg"] + r * out["E"]
    np.testing.assert_allclose(after, before, rtol=1e-14)
    # without q the same step deposits nothing
    p.irr = None
    out0, _ = orc.Oracle(p).implicit(f, star, dt)
    np.testing.assert_allclose(out0["Eg"] + r * out0["E"], f["Eg"] + r * f["E"], rtol=1e-14)
    assert np.all(out["Eg"] > out0["Eg"])


# ---------------------------------------------------------------------------
# absorption only
# ---------------------------------------------------------------------------

def test_absorption_only_rate_and_bounds(orc):
    n = (8, 1, 1)
    rng = np.random.default_rng(9)
    f = _random_fields(rng, (1, 1, 8))
    f["Eg"] *= 100.0                              # hot gas: would emit strongly
    one = [np.array([0.0, 1.0])] * 2
    p = _problem(n, 1, [_faces(8, 1.0)] + one, [[0, 0]] * 3, f, kP=2.0, kR=1.0, c_hat=3.0)
    p.c = 30.0
    star = {k: f[k] for k in ("E", "Fx", "Fy", "Fz")}
    p.absorb_only = 1
    r = p.c / p.c_hat
    for dt in (1e-2, 1e-1):
        out, _ = orc.Oracle(p).implicit(f, star, dt)
        assert np.all(out["E"] < f["E"])           # never emitted, only absorbed
        np.testing.assert_allclose(out["Eg"] + r * out["E"], f["Eg"] + r * f["E"], rtol=1e-14)
    # continuous limit: dE/dt = -c_hat kappa_P rho E
    dt = 1e-7
    out, _ = orc.Oracle(p).implicit(f, star, dt)
    rate = (out["E"] - f["E"]) / dt
    np.testing.assert_allclose(rate, -p.c_hat * 2.0 * f["rho"] * f["E"], rtol=1e-5)
    # the full coupling heats the radiation instead
    p.absorb_only = 0
    out, _ = orc.Oracle(p).implicit(f, star, 1e-2)
    assert np.all(out["E"] > f["E"])


# ---------------------------------------------------------------------------
# the shadow test (reduced grid)
# ---------------------------------------------------------------------------

def test_shadow_is_sharp_behind_the_spheroid(orc):
    p = I.make_shadow(nx=70, ny=20, absorb_only=1, t_end=1.5)
    r, cnt = orc.Oracle(p).run(p.fields, p.dt, p.steps)
    E = r["E"][0] / (p.a_rad * 6.0 ** 4)           # in units of the beam
    xc = 0.5 * (p.faces[0][1:] + p.faces[0][:-1])
    yc = 0.5 * (p.faces[1][1:] + p.faces[1][:-1])
    right = xc > 0.25
    shadow = E[np.ix_(yc < 0.035, right)]
    lit = E[np.ix_(yc > 0.12, right)]
    # lit: the beam attenuated by the background absorption 0.1 per unit length
    att = np.exp(-0.1 * (xc[right] + 0.5))
    assert np.all(np.abs(lit / att - 1) < 0.05), np.abs(lit / att - 1).max()
    assert shadow.max() < 0.02, shadow.max()
    # the edge of the shadow spans a few cells at x = 0.4
    col = E[:, np.argmin(np.abs(xc - 0.4))] / math.exp(-0.09)
    j10, j90 = np.argmax(col > 0.1), np.argmax(col > 0.9)
    assert 0 < j90 - j10 <= 4, (j10, j90)
    # inside the opaque spheroid the radiation is absorbed down to the floor
    assert cnt[0] > 0
