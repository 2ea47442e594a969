"""Pins of the oracle's multigroup M1 (one gray fluid per frequency group,
an (m+1)^2 implicit system, Sect. 2.3 and 2.8):

* the Planck fraction against adaptive quadrature of the Planck integrand
  (library routine), its limits, and group fractions summing to one;
* one group reduces to the gray system solved in closed form;
* groups with equal opacities aggregate to the gray system for the summed
  energy (independent of how the radiation is split between groups);
* a Planck spectrum in equilibrium with the gas is a fixed point;
* the whole run conserves E_g + (c / c_hat) sum_g E_g on a periodic box, and
  a one-group run equals the gray run.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2606_26268_amd import inputs as I


def _planck_quad(x):
    return quad(lambda t: t ** 3 / np.expm1(t), 0.0, x, epsabs=0.0, epsrel=1e-13, limit=200)[0] * 15 / np.pi ** 4


def test_planck_fraction_against_quadrature(orc):
    xs = np.concatenate([np.geomspace(1e-3, 60.0, 200), [0.999999, 1.0, 1.000001]])
    err = max(abs(orc.planck_cdf(x) - _planck_quad(x)) / _planck_quad(x) for x in xs)
    assert err < 1e-12, err
    assert orc.planck_cdf(0.0) == 0.0 and abs(orc.planck_cdf(200.0) - 1.0) < 1e-15
    # small-x limit: P(x) ~ (15 / pi^4) x^3 / 3
    assert abs(orc.planck_cdf(1e-4) / (15 / np.pi ** 4 * 1e-12 / 3) - 1) < 1e-4
    # Wien peak of the energy spectrum: x^3 / (e^x - 1) is largest at x = 2.8214...
    h = 1e-4
    d = [(orc.planck_cdf(x + h) - orc.planck_cdf(x - h)) / (2 * h) for x in (2.78, 2.8214393721, 2.86)]
    assert d[1] > d[0] and d[1] > d[2]


def test_group_fractions_sum_to_one(orc):
    edges = [0.5, 1.5, 3.0, 6.0, 12.0]
    for T in (0.1, 1.0, 3.7, 50.0):
        b = orc.group_fractions(edges, T)
        assert np.all(b >= 0) and abs(b.sum() - 1.0) < 1e-15
    # a hot gas puts its energy in the highest band, a cold one in the lowest
    assert orc.group_fractions(edges, 100.0)[-1] > 0.99 and orc.group_fractions(edges, 0.01)[0] > 0.99


def _gray_closed_form(orc, Es, Cv, T, kP, rho, dt, c_hat, c, a, S=0.0):
    """The gray 2x2 system in its cancellation-free closed form (pinned by
    its residuals in the implicit-step tests)."""
    E1, T1, _, _ = orc.implicit_cell(Es, Cv, T, kP, rho, dt, c_hat, c, a, S)
    return E1, T1


def test_one_group_is_the_gray_system(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        Es, Cv, T, kP, rho = np.exp(rng.normal(size=5))
        dt, c_hat = 10 ** rng.uniform(-4, -1), 10 ** rng.uniform(0, 2)
        c = c_hat * 10 ** rng.uniform(0, 2)
        S = rng.uniform(0, 1)
        x = orc.mg_cell([Es], Cv, T, [kP], rho, dt, c_hat, c, 1.0, [1.0], S)
        E1, T1 = _gray_closed_form(orc, Es, Cv, T, kP, rho, dt, c_hat, c, 1.0, S)
        assert abs(x[0] - E1) <= 1e-12 * E1 and abs(x[1] - T1) <= 1e-12 * T1


def test_equal_opacities_aggregate_to_gray(orc):
    rng = np.random.default_rng(2)
    edges = [0.7, 2.0, 4.5]
    for _ in range(100):
        Cv, T, kP, rho = np.exp(rng.normal(size=4))
        Es = np.exp(rng.normal(size=4))
        dt, c_hat, c = 0.05, 3.0, 30.0
        b = orc.group_fractions(edges, T)
        x = orc.mg_cell(Es, Cv, T, [kP] * 4, rho, dt, c_hat, c, 1.0, b)
        E1, T1 = _gray_closed_form(orc, Es.sum(), Cv, T, kP, rho, dt, c_hat, c, 1.0)
        assert abs(x[:4].sum() - E1) <= 1e-12 * E1 and abs(x[4] - T1) <= 1e-12 * T1


def test_planck_equilibrium_is_a_fixed_point(orc):
    edges = [0.7, 2.0, 4.5, 9.0]
    for T in (0.3, 1.0, 2.5):
        b = orc.group_fractions(edges, T)
        Es = b * T ** 4
        x = orc.mg_cell(Es, 1.5, T, [0.1, 1.0, 10.0, 100.0, 1e3], 1.0, 0.1, 5.0, 50.0, 1.0, b)
        assert np.allclose(x[:5], Es, rtol=1e-13) and abs(x[5] - T) <= 1e-13 * T


def _mg_problem(m, n=(12, 10, 8), seed=5):
    rng = np.random.default_rng(seed)
    faces = [I.uniform_faces(k, 0.0, 1.0) for k in n]
    p = I.make_random_state(I.CARTESIAN, n, 3, seed, faces, [[I.PERIODIC] * 2] * 3, fmax=0.7, c_hat=2.0)
    shape = p.fields["E"].shape
    scale = rng.uniform(0.2, 1.0, m)             # one factor per group keeps f <= 0.7
    for k in ("E", "Fx", "Fy", "Fz"):
        p.fields[k] = np.stack([p.fields[k] * scale[g] for g in range(m)])
    p.groups = dict(edges=list(np.geomspace(0.5, 8.0, m - 1)) if m > 1 else [],
                    kP=list(np.geomspace(0.2, 20.0, m)), kR=list(np.geomspace(0.5, 5.0, m)))
    p.opacity = dict(kind=I.OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.1)
    p.c = 20.0
    p.dt = 0.3 / (2.0 * sum(n))
    assert shape == p.fields["rho"].shape
    return p


def test_multigroup_run_conserves_the_rescaled_total(orc):
    p = _mg_problem(5)
    r, cnt = orc.Oracle(p).run_mg(p.fields, p.dt, 10)
    ratio = p.c / p.c_hat
    tot0 = p.fields["Eg"].sum() + ratio * p.fields["E"].sum()
    tot1 = r["Eg"].sum() + ratio * r["E"].sum()
    assert abs(tot1 - tot0) <= 1e-12 * tot0
    for q, k in enumerate(("Fx", "Fy", "Fz")):
        mom0 = p.fields["m" + k[1]].sum() + p.fields[k].sum() / p.c_hat
        mom1 = r["m" + k[1]].sum() + r[k].sum() / p.c_hat
        assert abs(mom1 - mom0) <= 1e-12 * (abs(p.fields[k]).sum() / p.c_hat)


def test_one_group_run_equals_gray_run(orc):
    p = _mg_problem(1)
    r, _ = orc.Oracle(p).run_mg(p.fields, p.dt, 6)
    q = _mg_problem(1)
    q.groups = None
    for k in ("E", "Fx", "Fy", "Fz"):
        q.fields[k] = np.ascontiguousarray(q.fields[k][0])
    q.opacity = dict(kind=I.OPAC_CONSTANT, kP=p.groups["kP"][0], kR=p.groups["kR"][0], sigma=0.1)
    g, _ = orc.Oracle(q).run(q.fields, q.dt, 6)
    for k in ("E", "Fx", "Fy", "Fz"):
        np.testing.assert_allclose(r[k][0], g[k], rtol=1e-12, atol=1e-14, err_msg=k)
    for k in ("mx", "my", "mz", "Eg"):
        np.testing.assert_allclose(r[k], g[k], rtol=1e-12, atol=1e-14, err_msg=k)


def test_multigroup_relaxes_towards_a_planck_spectrum(orc):
    """Uniform medium, no flux: the groups relax to b_g(T) a T^4 at the
    temperature fixed by the conserved total."""
    p = _mg_problem(4, n=(4, 4, 4), seed=9)
    for k in ("E", "Fx", "Fy", "Fz", "mx", "my", "mz"):
        p.fields[k][:] = 0.0
    p.fields["E"][:] = 1e-3
    p.fields["rho"][:] = 1.0
    p.fields["Eg"][:] = 1.5 * 2.0                 # T = 2, far hotter than the radiation
    p.c = p.c_hat = 1.0
    p.groups["kP"] = [50.0] * 4
    r, _ = orc.Oracle(p).run_mg(p.fields, 0.05, 400)
    T = r["Eg"][0, 0, 0] / 1.5
    b = orc.group_fractions(p.groups["edges"], T)
    Eg = r["E"][:, 0, 0, 0]
    assert np.allclose(Eg, b * T ** 4, rtol=1e-6), (Eg, b * T ** 4)
    # energy balance: 1.5 T + sum E = 1.5 * 2 + 4e-3
    assert abs(1.5 * T + Eg.sum() - (3.0 + 4e-3)) < 1e-12


def test_multigroup_absorption_only(orc):
    p = _mg_problem(3)
    p.absorb_only = 1
    o = orc.Oracle(p)
    r, _ = o.run_mg(p.fields, p.dt, 1)
    q = _mg_problem(3)
    q.absorb_only = 1
    q.groups = dict(q.groups, kP=[0.0] * 3)          # transport alone
    t, _ = orc.Oracle(q).run_mg(q.fields, q.dt, 1)
    for g in range(3):
        kP = p.groups["kP"][g]
        np.testing.assert_allclose(r["E"][g], t["E"][g] / (1 + p.dt * p.c_hat * kP * p.fields["rho"]), rtol=1e-14)
    ratio = p.c / p.c_hat
    np.testing.assert_allclose(r["Eg"] + ratio * r["E"].sum(axis=0), t["Eg"] + ratio * t["E"].sum(axis=0), rtol=1e-14)


def test_one_group_rk2_equals_gray_rk2(orc):
    """The multigroup second-order step with one group is the gray one."""
    p = _mg_problem(1)
    r, _ = orc.Oracle(p).run_mg(p.fields, p.dt, 4, rk2=True)
    q = _mg_problem(1)
    q.groups = None
    for k in ("E", "Fx", "Fy", "Fz"):
        q.fields[k] = np.ascontiguousarray(q.fields[k][0])
    q.opacity = dict(kind=I.OPAC_CONSTANT, kP=p.groups["kP"][0], kR=p.groups["kR"][0], sigma=0.1)
    g, _ = orc.Oracle(q).run(q.fields, q.dt, 4, rk2=True)
    for k in ("E", "Fx", "Fy", "Fz"):
        np.testing.assert_allclose(r[k][0], g[k], rtol=1e-12, atol=1e-14, err_msg=k)
    for k in ("mx", "my", "mz", "Eg"):
        np.testing.assert_allclose(r[k], g[k], rtol=1e-12, atol=1e-14, err_msg=k)


def test_multigroup_rk2_conserves_and_differs_from_euler(orc):
    """Each stage conserves E_g + (c / c_hat) sum_g E_g and m + sum_g F_g / c_hat
    on a periodic box, so their average does; and the averaged step is not
    the Euler step."""
    p = _mg_problem(4)
    r, _ = orc.Oracle(p).run_mg(p.fields, p.dt, 3, rk2=True)
    ratio = p.c / p.c_hat
    tot0 = p.fields["Eg"].sum() + ratio * p.fields["E"].sum()
    tot1 = r["Eg"].sum() + ratio * r["E"].sum()
    assert abs(tot1 - tot0) <= 1e-12 * tot0
    for q, k in enumerate(("Fx", "Fy", "Fz")):
        mom0 = p.fields["m" + k[1]].sum() + p.fields[k].sum() / p.c_hat
        mom1 = r["m" + k[1]].sum() + r[k].sum() / p.c_hat
        assert abs(mom1 - mom0) <= 1e-12 * (abs(p.fields[k]).sum() / p.c_hat)
    e, _ = orc.Oracle(p).run_mg(p.fields, p.dt, 3)
    assert np.abs(e["E"] - r["E"]).max() > 1e-9 * np.abs(r["E"]).max()
