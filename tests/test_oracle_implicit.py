"""Pins of the oracle's implicit radiation-matter step (Sect. 2.8) and of its
opacity sources.

References independent of the oracle's own algebra: the discrete equations
the paper starts from (Eqs. source_discrete1 / internal with the T^4
linearisation) checked as residuals; the radiative-equilibrium limit found
as the root of a quartic by a library polynomial solver; exact fixed points;
conservation of the rescaled totals (Sect. 2.7); the flux damping law
(Eq. source_discrete2); bilinear interpolation special cases and bounds.
"""
import math

import numpy as np
import pytest

from paper_2606_26268_amd import inputs as I


def test_implicit_cell_solves_the_discrete_equations(orc):
    rng = np.random.default_rng(0)
    for _ in range(500):
        Es = math.exp(rng.normal())
        rho = math.exp(rng.normal())
        Cv = rho / (2.0 / 3.0)
        T = math.exp(0.3 * rng.normal())
        kP = math.exp(2 * rng.normal())
        dt = 10 ** rng.uniform(-6, -1)
        c_hat = 10 ** rng.uniform(0, 2)
        c = c_hat * 10 ** rng.uniform(0, 3)
        a = 1.0
        E1, T1, E1c, T1c = orc.implicit_cell(Es, Cv, T, kP, rho, dt, c_hat, c, a)
        lin4 = 4 * T1 * T ** 3 - 3 * T ** 4          # linearised (T^{n+1})^4
        gr = dt * c_hat * kP * rho                     # dt / t_abs,red
        g = dt * c * kP * rho                          # dt / t_abs
        r1 = E1 * (1 + gr) - gr * a * lin4 - Es        # Eq. source_discrete1
        r2 = Cv * T1 + g * a * lin4 - g * E1 - Cv * T  # discretised Eq. internal
        # scales: sum of magnitudes of every term, the linearised T^4 expanded
        s1 = abs(E1) * (1 + gr) + gr * a * (4 * T1 * T ** 3 + 3 * T ** 4) + abs(Es)
        s2 = Cv * abs(T1) + g * a * (4 * T1 * T ** 3 + 3 * T ** 4) + g * abs(E1) + Cv * T
        assert abs(r1) <= 1e-14 * s1
        assert abs(r2) <= 1e-14 * s2
        assert E1 > 0 and T1 > 0
        # literal Cramer agrees within its own rounding
        assert abs(E1 - E1c) <= 1e-9 * (abs(E1) + gr * a * T ** 4)


def test_equilibrium_is_a_fixed_point(orc):
    for T in (0.5, 1.0, 3.0):
        E1, T1, _, _ = orc.implicit_cell(T ** 4, 1.5, T, 5.0, 1.0, 0.1, 10.0, 1000.0)
        assert abs(E1 - T ** 4) <= 4e-16 * T ** 4
        assert abs(T1 - T) <= 4e-16 * T


def _uniform_cell(E0, T0, kP, c_hat, c, sigma=0.0, F=(0.0, 0.0, 0.0)):
    p = I.make_uniform(I.CARTESIAN, (4, 1, 1), 1, E=E0, F=F, kP=kP, kR=kP, sigma=sigma, c_hat=c_hat)
    p.c = c
    p.fields["Eg"][:] = 1.0 * T0 / (p.gamma - 1)
    return p


def test_relaxation_to_radiative_equilibrium(orc):
    """E0 = 2, T0 = 1, C_v = 1.5, c = c_hat: the limit solves
    C_v T + (c/c_hat) a T^4 = C_v T0 + (c/c_hat) E0 (roots of a quartic)."""
    p = _uniform_cell(2.0, 1.0, 5.0, 10.0, 10.0)
    o = orc.Oracle(p)
    st = p.fields
    Es, Ts = [2.0], [1.0]
    for _ in range(400):
        st, cnt = o.run(st, 0.01, 1)
        Es.append(st["E"][0, 0, 0])
        Ts.append(st["Eg"][0, 0, 0] / 1.5)
    roots = np.roots([1.0, 0.0, 0.0, 1.5, -(1.5 + 2.0)])
    Teq = max(r.real for r in roots if abs(r.imag) < 1e-12 and r.real > 0)
    assert abs(Teq - 1.1534154418) < 1e-9
    assert abs(Ts[-1] - Teq) < 1e-12 and abs(Es[-1] - Teq ** 4) < 1e-12
    # monotone approach without overshoot
    assert all(np.diff(Es) <= 1e-15) and all(np.diff(Ts) >= -1e-15)
    assert min(Es) >= Teq ** 4 - 1e-12 and max(Ts) <= Teq + 1e-12


def test_flux_damping_closed_form(orc):
    dt, c_hat, kR, sigma, rho = 0.01, 7.0, 2.0, 3.0, 1.0
    p = _uniform_cell(1.0, 1.0, 0.0, c_hat, c_hat, sigma=sigma, F=(0.3, -0.2, 0.1))
    p.opacity = dict(kind=I.OPAC_CONSTANT, kP=0.0, kR=kR, sigma=sigma)
    o = orc.Oracle(p)
    star = {k: p.fields[k].copy() for k in ("E", "Fx", "Fy", "Fz")}
    out, cnt = o.implicit(p.fields, star, dt)
    d = 1 + dt * c_hat * (kR + sigma) * rho       # Eq. source_discrete2
    for k, v in (("Fx", 0.3), ("Fy", -0.2), ("Fz", 0.1)):
        assert abs(out[k][0, 0, 0] - v / d) <= abs(np.spacing(v / d))
        m = {"Fx": "mx", "Fy": "my", "Fz": "mz"}[k]
        assert abs(out[m][0, 0, 0] + (v / d - v) / c_hat) < 1e-16


def test_stiff_reduced_speed_of_light_conserves(orc):
    """c / c_hat = 1e4: the gas update amplifies the radiation change by 1e4;
    the cancellation-free solve must still conserve E_g + (c/c_hat) E."""
    rng = np.random.default_rng(5)
    p = I.make_random_state(I.CARTESIAN, (64, 1, 1), 1, 3,
                            [I.uniform_faces(64, 0, 1), np.array([0., 1.]), np.array([0., 1.])],
                            [[I.PERIODIC] * 2] * 3, fmax=0.5, c_hat=1.0,
                            opacity=dict(kind=I.OPAC_CONSTANT, kP=50.0, kR=10.0, sigma=0.0))
    p.c = 1e4
    o = orc.Oracle(p)
    star = {k: p.fields[k] * (1 + 0.1 * rng.random(p.fields[k].shape)) for k in ("E", "Fx", "Fy", "Fz")}
    out, cnt = o.implicit(p.fields, star, 1e-3)
    r = p.c / p.c_hat
    before = p.fields["Eg"] + r * star["E"]
    after = out["Eg"] + r * out["E"]
    assert np.abs(after - before).max() <= 4e-16 * np.abs(before).max() * 4
    assert cnt[3] == 0


def test_absorption_free_step_is_identity(orc):
    p = _uniform_cell(1.3, 0.7, 0.0, 5.0, 5.0, F=(0.2, 0.1, 0.0))
    o = orc.Oracle(p)
    star = {k: p.fields[k].copy() for k in ("E", "Fx", "Fy", "Fz")}
    out, cnt = o.implicit(p.fields, star, 0.1)
    for k in ("E", "Fx", "Fy", "Fz", "Eg", "mx"):
        assert np.array_equal(out[k], p.fields[k])


# ----------------------------------------------------------------------------
# opacity
# ----------------------------------------------------------------------------

def _table_problem(kp, kr, lr=(0.0, 127.0), lt=(0.0, 127.0), off=(0.0, 0.0)):
    p = I.make_uniform(I.CARTESIAN, (2, 1, 1), 1)
    nt, nr = kp.shape
    p.opacity = dict(kind=I.OPAC_TABLE, nr=nr, nt=nt, lr0=lr[0], lr1=lr[1], lt0=lt[0], lt1=lt[1],
                     lr_off=off[0], lt_off=off[1], log10_kP=kp, log10_kR=kr, sigma=0.0)
    return p


def test_table_reproduces_linear_functions_and_nodes(orc):
    """Integer node grid with integer-valued (exact in binary32) linear data:
    bilinear interpolation must return the linear function everywhere."""
    j, i = np.meshgrid(np.arange(128.0), np.arange(128.0), indexing="ij")
    kp = (-3.0 + 0.125 * i - 0.25 * j).astype(np.float32)
    kr = (1.0 - 0.5 * i + 0.0625 * j).astype(np.float32)
    o = orc.Oracle(_table_problem(kp, kr))
    rng = np.random.default_rng(0)
    lr = rng.uniform(0, 127, 2000)
    lt = rng.uniform(0, 127, 2000)
    P, R = o.opacity(10 ** lr, 10 ** lt)
    np.testing.assert_allclose(np.log10(P), -3.0 + 0.125 * lr - 0.25 * lt, atol=1e-12)
    np.testing.assert_allclose(np.log10(R), 1.0 - 0.5 * lr + 0.0625 * lt, atol=1e-12)
    # node values and clamping outside the axes
    P, R = o.opacity(10.0 ** np.array([3.0, -5.0, 200.0]), 10.0 ** np.array([7.0, 50.0, 200.0]))
    np.testing.assert_allclose(np.log10(P), [kp[7, 3], kp[50, 0], kp[127, 127]], atol=1e-12)


def test_synthetic_table_close_to_its_smooth_function(orc):
    """Bilinear error <= h^2/8 * max|d2/dlT2| plus binary32 rounding."""
    tab = I.make_table()
    p = I.make_uniform(I.CARTESIAN, (2, 1, 1), 1)
    p.opacity = tab
    o = orc.Oracle(p)
    rng = np.random.default_rng(1)
    lr = rng.uniform(-12, 0, 20000)
    lt = rng.uniform(2, 6, 20000)
    P, R = o.opacity(10 ** (lr + 5.0), 10 ** (lt - 4.0))
    fp, fr = I.table_log10_kappa(lr, lt)
    h = 4.0 / 127
    g = np.linspace(2, 6, 40001)
    for got, smooth, col in ((P, fp, 0), (R, fr, 1)):
        curv = np.abs(np.gradient(np.gradient(I.table_log10_kappa(0 * g, g)[col], g), g)).max()
        bound = h * h / 8 * curv * 1.01 + 2e-6     # interpolation + binary32 rounding
        assert np.abs(np.log10(got) - smooth).max() < bound


def test_power_law_opacity(orc):
    p = I.make_uniform(I.CARTESIAN, (2, 1, 1), 1)
    p.opacity = dict(kind=I.OPAC_POWERLAW, k0=0.1, rho0=2.0, alpha=1.0, T0=3.0, beta=-3.5, sigma=0.0)
    o = orc.Oracle(p)
    P, R = o.opacity(np.array([2.0, 4.0, 2.0]), np.array([3.0, 3.0, 6.0]))
    np.testing.assert_allclose(P, [0.1, 0.2, 0.1 * 2 ** -3.5], rtol=1e-15)
    np.testing.assert_allclose(R, P, rtol=0)
