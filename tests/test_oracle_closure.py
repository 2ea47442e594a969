"""Pins of the oracle's closure, signal speeds, fluxes, HLL, slope and face fix.

Each check compares the oracle with something the paper or the mathematics
fixes independently of the oracle's own formulas:

* the Levermore closure is exact for a Lorentz-boosted isotropic intensity
  (Sect. 2.1), so moments integrated numerically from I ~ (1 - beta mu)^-4
  must reproduce f and the Eddington factor;
* the Sect. 2.6 speeds must be the extreme eigenvalues of the Jacobian of the
  flux (numerical differentiation + a library eigen-solver), and the middle
  ones the contact speed lambda_2;
* printed limits (f -> 0 and f -> 1) and brute-force bounds |lambda| <= 1;
* HLL special cases (upwind for a free-streaming state, Rusanov for
  symmetric speeds, consistency, the optical-depth clamp).
"""
import math

import numpy as np
import pytest


def boosted_moments(beta):
    """E, F, P_par, P_perp of I(mu) = (1 - beta mu)^-4 (per 2 pi), integrated
    by 400-point Gauss-Legendre quadrature (converged to rounding for
    beta <= 0.97: the integrand's pole sits at mu = 1/beta)."""
    mu, wq = np.polynomial.legendre.leggauss(400)
    w = wq * (1.0 - beta * mu) ** -4
    return w.sum(), (w * mu).sum(), (w * mu * mu).sum(), (w * 0.5 * (1 - mu * mu)).sum()


def test_xi_limits(orc):
    assert abs(orc.xi(0.0) - 1.0 / 3.0) <= np.spacing(1.0 / 3.0)
    assert orc.xi(1.0) == 1.0


@pytest.mark.parametrize("beta", [0.0, 0.05, 0.2, 0.4, 0.6, 0.8, 0.9, 0.97])
@pytest.mark.parametrize("direction", [(1, 0, 0), (0, 1, 0), (0.6, 0, 0.8), (0.48, 0.6, 0.64)])
def test_closure_matches_boosted_isotropic_intensity(orc, beta, direction):
    E, F, Pp, Pt = boosted_moments(beta)
    n = np.array(direction, dtype=float)
    n /= np.linalg.norm(n)
    f, xi, D = orc.eddington(1.0, F / E * n)
    assert abs(f - F / E) < 1e-14
    assert abs(xi - Pp / E) < 1e-12
    # full tensor: P = P_par n n + P_perp (I - n n), normalised by E
    D_ref = (Pp / E) * np.outer(n, n) + (Pt / E) * (np.eye(3) - np.outer(n, n))
    np.testing.assert_allclose(D, D_ref, atol=1e-12, rtol=0)


def test_eddington_trace_and_eigen(orc):
    rng = np.random.default_rng(0)
    for _ in range(200):
        E = math.exp(rng.normal())
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        F = rng.uniform(0, 1) * E * n
        f, xi, D = orc.eddington(E, F)
        assert abs(np.trace(D) - 1.0) <= 4 * np.finfo(float).eps
        np.testing.assert_allclose(D @ n, xi * n, atol=1e-15)
        t = np.cross(n, [0.3, -0.2, 0.9])
        t /= np.linalg.norm(t)
        np.testing.assert_allclose(D @ t, 0.5 * (1 - xi) * t, atol=1e-15)


def test_speed_limits(orc):
    rng = np.random.default_rng(1)
    for d in range(3):
        for _ in range(20):
            lm, lp = orc.speeds(2.0, [0, 0, 0], d)
            assert abs(lm + 1 / math.sqrt(3)) < 1e-15 and abs(lp - 1 / math.sqrt(3)) < 1e-15
            n = rng.normal(size=3)
            n /= np.linalg.norm(n)
            F = 3.0 * n
            E = math.sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2])   # f == 1 exactly
            lm, lp = orc.speeds(E, F, d)     # f = 1: both -> cos(theta)
            assert abs(lm - F[d] / E) < 1e-15 and abs(lp - F[d] / E) < 1e-15
    # near f = 1 the speeds are square-root sensitive: f = 1 - eps moves them
    # by O(sqrt(eps)); an inherent conditioning of the formula, bounded here
    lm, lp = orc.speeds(1.0, [1.0 - 1e-12, 0, 0], 1)
    assert abs(lm) < 3e-6 and abs(lp) < 3e-6


def _jacobian(orc, U, d, h=1e-6):
    J = np.zeros((4, 4))
    for b in range(4):
        dU = np.zeros(4)
        dU[b] = h * U[0]
        J[:, b] = (orc.flux(U[0] + dU[0], U[1:] + dU[1:], d) -
                   orc.flux(U[0] - dU[0], U[1:] - dU[1:], d)) / (2 * h * U[0])
    return J


def test_speeds_are_flux_jacobian_eigenvalues(orc):
    rng = np.random.default_rng(2)
    for _ in range(60):
        E = math.exp(rng.normal())
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        f = rng.uniform(0.05, 0.95)
        U = np.concatenate([[E], f * E * n])
        d = int(rng.integers(0, 3))
        ev = np.sort(np.linalg.eigvals(_jacobian(orc, U, d)).real)
        lm, lp = orc.speeds(E, U[1:], d)
        assert abs(ev[0] - lm) < 1e-6 and abs(ev[-1] - lp) < 1e-6
        # the two middle eigenvalues are the contact speed (3 xi - 1) cos / (2 f)
        lam2 = (3 * orc.xi(f) - 1) * n[d] / (2 * f)
        np.testing.assert_allclose(ev[1:3], [lam2, lam2], atol=2e-5)


def test_speeds_bounded_brute_force(orc):
    worst = 0.0
    for f in np.linspace(0, 1, 1001)[::10]:
        for mu in np.linspace(-1, 1, 1001)[::5]:
            s = math.sqrt(max(0.0, 1 - mu * mu))
            lm, lp = orc.speeds(1.0, [f * mu, f * s, 0.0], 0)
            worst = max(worst, abs(lm), abs(lp))
            assert lm <= lp
    assert worst <= 1.0


def test_hll_free_streaming_is_upwind(orc):
    UL = np.array([2.0, 2.0, 0.0, 0.0])     # f = 1 along +x
    UR = np.array([0.5, 0.5, 0.0, 0.0])
    out, SL, SR = orc.hll(UL, UR, 0, tau=0.0, c_hat=3.0)
    assert SL == 0.0 and abs(SR - 1.0) < 1e-15
    np.testing.assert_allclose(out, 3.0 * np.array([2.0, 2.0, 0.0, 0.0]), rtol=2e-16, atol=0)


def test_hll_consistency_and_rusanov(orc):
    rng = np.random.default_rng(3)
    for _ in range(50):
        E = math.exp(rng.normal())
        F = rng.uniform(0, 0.9) * E * (lambda v: v / np.linalg.norm(v))(rng.normal(size=3))
        U = np.concatenate([[E], F])
        d = int(rng.integers(0, 3))
        out, _, _ = orc.hll(U, U, d, c_hat=2.0)
        np.testing.assert_allclose(out, 2.0 * orc.flux(E, F, d), rtol=1e-14, atol=1e-14)
    # isotropic states on both sides: speeds -+1/sqrt(3) -> Rusanov flux
    UL = np.array([2.0, 0, 0, 0])
    UR = np.array([1.0, 0, 0, 0])
    out, SL, SR = orc.hll(UL, UR, 0)
    s = 1 / math.sqrt(3)
    ref = 0.5 * (orc.flux(2.0, [0, 0, 0], 0) + orc.flux(1.0, [0, 0, 0], 0)) - 0.5 * s * (UR - UL)
    np.testing.assert_allclose(out, ref, rtol=1e-15, atol=1e-15)


def test_hll_optical_depth_clamp(orc):
    UL = np.array([2.0, 0, 0, 0])
    UR = np.array([1.0, 0, 0, 0])
    tau = 50.0
    out, SL, SR = orc.hll(UL, UR, 0, tau=tau)
    lim = 4 / (3 * tau)
    assert abs(SL + lim) < 1e-16 and abs(SR - lim) < 1e-16
    ref = 0.5 * (orc.flux(2.0, [0, 0, 0], 0) + orc.flux(1.0, [0, 0, 0], 0)) - 0.5 * lim * (UR - UL)
    np.testing.assert_allclose(out, ref, rtol=1e-15, atol=1e-15)
    # thin cells leave the speeds untouched
    out2, SL2, SR2 = orc.hll(UL, UR, 0, tau=0.1)
    assert abs(SL2 + 1 / math.sqrt(3)) < 1e-15


def test_vanleer_cases(orc):
    assert orc.vanleer(1.0, 1.0) == 1.0
    assert orc.vanleer(2.0, -1.0) == 0.0
    assert orc.vanleer(0.0, 3.0) == 0.0
    assert abs(orc.vanleer(1.0, 3.0) - 1.5) < 1e-16
    # limited slope never exceeds twice the smaller one-sided slope
    rng = np.random.default_rng(4)
    for a, b in rng.normal(size=(500, 2)):
        s = orc.vanleer(a, b)
        if a * b > 0:
            assert abs(s) <= 2 * min(abs(a), abs(b)) + 1e-15
            assert min(a, b) <= s <= max(a, b)


def test_ffix_branches(orc):
    # face f larger than centre f and <= 1: kept
    br, E, F = orc.ffix(1.0, [0.6, 0, 0], 1.0, [0.5, 0, 0])
    assert br == 0 and F[0] == 0.6
    # tie f_face == f_centre: the 'otherwise' branch (strict '>')
    br, E, F = orc.ffix(2.0, [0.0, 1.0, 0], 1.0, [0.5, 0, 0])
    assert br == 1 and np.allclose(F, [1.0, 0, 0])
    # face f > 1: rescaled to the centre's f along the centre direction
    br, E, F = orc.ffix(1.0, [1.2, 0, 0], 2.0, [1.0, 0.2, 0])
    assert br == 1 and np.allclose(F, [0.5, 0.1, 0])
    # non-positive face energy: flat state
    br, E, F = orc.ffix(-1.0, [0.1, 0, 0], 2.0, [1.0, 0.2, 0])
    assert br == 2 and E == 2.0 and np.allclose(F, [1.0, 0.2, 0])


def test_alternative_face_treatments(orc):
    """PLUTO flat fallback and simple clip (Sect. 2.5 / 3.2) act only when
    |R(F)| > R(E); clip restores f = 1 along R(F), PLUTO the cell state."""
    for recon in (1, 2):
        br, E, F = orc.face_fix(recon, 1.0, [0.6, 0.2, 0.0], 2.0, [1.0, 0.2, 0.0])
        assert br == 0 and np.allclose(F, [0.6, 0.2, 0.0]) and E == 1.0
    br, E, F = orc.face_fix(1, 1.0, [1.2, 0.5, 0.0], 2.0, [1.0, 0.2, 0.0])
    assert br == 2 and E == 2.0 and np.allclose(F, [1.0, 0.2, 0.0])
    br, E, F = orc.face_fix(2, 1.0, [1.2, 0.5, 0.0], 2.0, [1.0, 0.2, 0.0])
    assert br == 1 and E == 1.0 and abs(np.linalg.norm(F) - 1.0) < 1e-15
    assert abs(F[1] / F[0] - 0.5 / 1.2) < 1e-15


def test_lax_friedrichs_flux(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        U = np.concatenate([[math.exp(rng.normal())], 0.5 * rng.uniform(-1, 1, 3)])
        d = int(rng.integers(0, 3))
        np.testing.assert_allclose(orc.lf(U, U, d, c_hat=3.0), 3.0 * orc.flux(U[0], U[1:], d), rtol=1e-14, atol=1e-14)
    # symmetric speeds: LF and HLL coincide (both Rusanov)
    UL, UR = np.array([2.0, 0, 0, 0]), np.array([1.0, 0, 0, 0])
    np.testing.assert_allclose(orc.lf(UL, UR, 0), orc.hll(UL, UR, 0)[0], rtol=1e-15, atol=1e-15)
    # one-sided speeds: LF adds dissipation HLL (upwind) does not
    UL, UR = np.array([2.0, 2.0, 0, 0]), np.array([1.0, 1.0, 0, 0])
    lf, hll = orc.lf(UL, UR, 0), orc.hll(UL, UR, 0)[0]
    np.testing.assert_allclose(hll, [2.0, 2.0, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(lf, 0.5 * (orc.flux(2.0, [2, 0, 0], 0) + orc.flux(1.0, [1, 0, 0], 0)) - 0.5 * (UR - UL),
                               rtol=1e-15)
