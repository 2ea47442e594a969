"""Seeded synthetic workloads for the gray M1 radiation step.

This module only *describes* inputs: grids (face coordinates), initial fields,
physical constants, the opacity table contents and MLP training samples.  It
holds none of the scheme's arithmetic (no closure, fluxes, geometry factors,
reconstruction or source solve), so both the HIP path and the CPU oracle can
be fed from it without sharing any of the method.  The time step is part of a
workload's definition and reaches both sides as an input: a stated value, or
on uniform Cartesian grids the Courant number over c_hat times the summed
inverse cell widths of the active directions; the method's general rule for
any grid (m1_max_dt in the library, m1o_max_dt in the oracle) is not here.

Every array is float64 unless noted, shaped (nz, ny, nx) with x fastest; the
first index direction of the grid ("d = 0") is x / R / r, "d = 1" is y / phi /
theta, "d = 2" is z / z / phi for Cartesian / cylindrical / spherical grids.

Workloads (sizes follow the scheme's performance section and the benchmark
definitions; numbers are code units with a_R = 1, c = c_hat):

* ``c0``  1D Cartesian, 256 cells on [0,1) periodic, Gaussian pulse in E.
* ``c1``  3D Cartesian 128^3 periodic, log-normal density, random F.
* ``c2``  same recipe at 256^3.
* ``c3``  3D spherical 192x96x192, log r in [1,100], tabulated opacity.
* ``c4``  ``c3`` with an MLP opacity surrogate.
* shock tubes, oblique beam, pulses and diffusion problems used by tests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CARTESIAN, CYLINDRICAL, SPHERICAL = 0, 1, 2
PERIODIC, OUTFLOW, REFLECT, FIXED = 0, 1, 2, 3
OPAC_CONSTANT, OPAC_POWERLAW, OPAC_TABLE, OPAC_MLP = 0, 1, 2, 3

FIELD_NAMES = ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")


@dataclass
class Problem:
    """One synthetic workload: grid, constants, opacity source and fields."""

    name: str
    geometry: int
    ndim: int
    n: tuple  # (n0, n1, n2) interior cells along d = 0, 1, 2
    faces: list  # three float64 arrays of length n[d] + 1
    bc: list  # [[lo, hi]] * 3
    c_hat: float
    c: float
    a_rad: float = 1.0
    gamma: float = 5.0 / 3.0
    e_floor: float = 1e-30
    opacity: dict = field(default_factory=dict)
    fields: dict = field(default_factory=dict)
    dt: float = 0.0
    steps: int = 1
    recon: int = 0      # 0 f-preserving, 1 PLUTO flat, 2 simple clip
    riemann: int = 0    # 0 HLL, 1 Lax-Friedrichs-Rusanov
    limiter: int = 0    # 0 PLM with the van Leer slope, 1 LimO3
    bc_state: list = None   # [[lo, hi]] * 3 ghost (E, Fx, Fy, Fz) of FIXED sides
    irr: object = None      # per-cell irradiation heating -div F_irr (float64), or None
    absorb_only: int = 0    # 1: absorption without emission
    groups: dict = None     # multigroup: dict(edges=[m-1], kP=[m], kR=[m]); E, F get a leading group axis

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def ncells(self):
        return int(self.n[0] * self.n[1] * self.n[2])


# ----------------------------------------------------------------------------
# random fields
# ----------------------------------------------------------------------------

def _kmag(shape):
    ks = [np.fft.fftfreq(s) * s for s in shape]
    kk = np.meshgrid(*ks, indexing="ij")
    return np.sqrt(sum(k * k for k in kk))


def grf_from_white(white, slope):
    """Filter white noise by |k|^slope (k = 0 removed) -> zero-mean field.

    Power spectrum P(k) = |k|^(2*slope) in the sense of the 3D power; the
    result is returned with unit variance.
    """
    k = _kmag(white.shape)
    filt = np.zeros_like(k)
    nz = k > 0
    filt[nz] = k[nz] ** slope
    g = np.fft.ifftn(np.fft.fftn(white) * filt).real
    g -= g.mean()
    return g / g.std()


def uniform_faces(n, lo, hi):
    return lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n


def _cart_faces(n, lo=0.0, hi=1.0):
    return [uniform_faces(n[d], lo, hi) if n[d] > 1 else np.array([lo, hi])
            for d in range(3)]


def _zeros(shape):
    return {k: np.zeros(shape) for k in FIELD_NAMES}


def _random_flux(rng, E, amp, shape):
    """|F| = amp * u * E with u ~ U[0,1) and an isotropic direction."""
    u = rng.random(shape)
    cth = rng.uniform(-1.0, 1.0, shape)
    phi = rng.uniform(0.0, 2.0 * np.pi, shape)
    sth = np.sqrt(1.0 - cth * cth)
    mag = amp * u * E
    return mag * sth * np.cos(phi), mag * sth * np.sin(phi), mag * cth


# ----------------------------------------------------------------------------
# benchmark workloads
# ----------------------------------------------------------------------------

def make_c0():
    """1D periodic Gaussian pulse, constant kappa_abs = 10, c_hat = 10."""
    n = (256, 1, 1)
    faces = _cart_faces(n)
    x = 0.5 * (faces[0][1:] + faces[0][:-1])
    f = _zeros((1, 1, 256))
    f["E"][:] = 1.0 + np.exp(-((x - 0.5) ** 2) / (2 * 0.05 ** 2))
    f["rho"][:] = 1.0
    gamma = 5.0 / 3.0
    f["Eg"][:] = 1.0 * 1.0 / (gamma - 1.0)
    return Problem("c0", CARTESIAN, 1, n, faces, [[PERIODIC] * 2] * 3,
                   c_hat=10.0, c=10.0, gamma=gamma,
                   opacity=dict(kind=OPAC_CONSTANT, kP=10.0, kR=10.0, sigma=0.0),
                   fields=f, dt=1.5625e-4, steps=100)


def make_turbulent_box(N, seed, dt, steps, name):
    """Log-normal density, smooth T, Mach-0.5 velocity, E = aT^4, random F."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (N, N, N)
    w_rho = rng.standard_normal(shape)
    w_T = rng.standard_normal(shape)
    w_v = [rng.standard_normal(shape) for _ in range(3)]
    g_rho = grf_from_white(w_rho, -1.0)
    g_T = grf_from_white(w_T, -2.0)
    g_T /= np.abs(g_T).max()
    v = [grf_from_white(w, -2.0) for w in w_v]
    vrms = math.sqrt(float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))
    v = [vi * (0.5 / vrms) for vi in v]
    rho = np.exp(g_rho - 0.5)
    T = 1.0 + 0.3 * g_T
    a, gamma = 1.0, 5.0 / 3.0
    E = a * T ** 4
    Fx, Fy, Fz = _random_flux(rng, E, 0.5, shape)
    f = dict(E=E, Fx=Fx, Fy=Fy, Fz=Fz, rho=rho,
             mx=rho * v[0], my=rho * v[1], mz=rho * v[2],
             Eg=rho * T / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    n = (N, N, N)
    return Problem(name, CARTESIAN, 3, n, _cart_faces(n), [[PERIODIC] * 2] * 3,
                   c_hat=20.0, c=20.0, gamma=gamma,
                   opacity=dict(kind=OPAC_CONSTANT, kP=1.0, kR=1.0, sigma=0.5),
                   fields=f, dt=dt, steps=steps)


def make_c1():
    return make_turbulent_box(128, 1, 5.2083e-5, 50, "c1")


def make_c2():
    return make_turbulent_box(256, 1, 2.6041e-5, 100, "c2")


# Synthetic opacity table: Kramers-like power law in (rho, T) plus three
# Gaussian bumps in log T; 128 x 128 nodes including both axis endpoints.
TABLE_NR, TABLE_NT = 128, 128
TABLE_LR = (-12.0, 0.0)
TABLE_LT = (2.0, 6.0)
TABLE_OFFSETS = (-5.0, 4.0)  # lookup at (log10 rho - 5, log10 T + 4)
_BUMP_MU = (3.0, 4.0, 5.0)
_BUMP_W = (0.5, 0.6, 0.5)
_BUMP_AP = (0.3, -0.25, 0.2)
_BUMP_AR = (0.2, 0.3, -0.25)


def table_log10_kappa(lr, lt):
    """Smooth function sampled into the table (float64): (log10 kP, log10 kR)."""
    lr = np.asarray(lr, dtype=np.float64)
    lt = np.asarray(lt, dtype=np.float64)
    base = (lr + 5.0) - 3.5 * (lt - 4.0)
    bp = sum(a * np.exp(-((lt - m) ** 2) / (2 * w * w)) for a, m, w in zip(_BUMP_AP, _BUMP_MU, _BUMP_W))
    br = sum(a * np.exp(-((lt - m) ** 2) / (2 * w * w)) for a, m, w in zip(_BUMP_AR, _BUMP_MU, _BUMP_W))
    return 1.0 + base + bp, 0.7 + base + br


def make_table(nr=TABLE_NR, nt=TABLE_NT):
    """Return dict with float32 [nT][nrho] arrays of log10 kappa_P and kappa_R
    (the benchmark's 128 x 128 nodes by default; other node counts sample the
    same function over the same axes)."""
    lr = TABLE_LR[0] + (TABLE_LR[1] - TABLE_LR[0]) * np.arange(nr) / (nr - 1)
    lt = TABLE_LT[0] + (TABLE_LT[1] - TABLE_LT[0]) * np.arange(nt) / (nt - 1)
    LT, LR = np.meshgrid(lt, lr, indexing="ij")
    kp, kr = table_log10_kappa(LR, LT)
    return dict(kind=OPAC_TABLE, nr=nr, nt=nt,
                lr0=TABLE_LR[0], lr1=TABLE_LR[1], lt0=TABLE_LT[0], lt1=TABLE_LT[1],
                lr_off=TABLE_OFFSETS[0], lt_off=TABLE_OFFSETS[1],
                log10_kP=np.ascontiguousarray(kp.astype(np.float32)),
                log10_kR=np.ascontiguousarray(kr.astype(np.float32)),
                sigma=0.0)


def spherical_faces(nr, nth, nph, r0=1.0, r1=100.0):
    lr0, lr1 = math.log10(r0), math.log10(r1)
    r = 10.0 ** (lr0 + (lr1 - lr0) * np.arange(nr + 1) / nr)
    th = np.pi * np.arange(nth + 1) / nth
    ph = 2.0 * np.pi * np.arange(nph + 1) / nph
    return [r, th, ph]


def make_c3(nr=192, nth=96, nph=192, seed=3, steps=100, dt=1.0435e-5, name="c3"):
    """Spherical stratified box with a perturbed r^-2 density and r^-1/2 T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nph, nth, nr)
    w = rng.standard_normal(shape)
    g = grf_from_white(w, -1.0)
    faces = spherical_faces(nr, nth, nph)
    rc = 0.5 * (faces[0][1:] + faces[0][:-1])
    R = np.broadcast_to(rc[None, None, :], shape)
    rho = R ** -2 * np.exp(0.5 * g - 0.125)
    T = R ** -0.5
    a, gamma = 1.0, 5.0 / 3.0
    E = a * T ** 4
    Fx, Fy, Fz = _random_flux(rng, E, 0.5, shape)
    z = np.zeros(shape)
    f = dict(E=np.ascontiguousarray(E), Fx=Fx, Fy=Fy, Fz=Fz, rho=np.ascontiguousarray(rho),
             mx=z.copy(), my=z.copy(), mz=z.copy(), Eg=np.ascontiguousarray(rho * T / (gamma - 1.0)))
    bc = [[OUTFLOW, OUTFLOW], [OUTFLOW, OUTFLOW], [PERIODIC, PERIODIC]]
    return Problem(name, SPHERICAL, 3, (nr, nth, nph), faces, bc,
                   c_hat=20.0, c=20.0, gamma=gamma, opacity=make_table(),
                   fields=f, dt=dt, steps=steps)


def make_c4(**kw):
    p = make_c3(name="c4", **kw)
    p.opacity = dict(make_table(), kind=OPAC_MLP)
    return p


def make_pulse3d(N=256, dx=0.5, steps=100, cfl=0.4):
    """The optically thin radiation pulse the scheme's performance section
    times (the Sect. 3.4 pulse on a 3D Cartesian grid), in units a T0^4 = 1:
    N^3 cells of width dx centred on the origin, periodic; radiation at
    T_r = 1 + 100 exp(-r^2 / 25) (w = 5), i.e. E = T_r^4, F = 0; gas at rest
    with rho = 1 and T = 1; no absorption (kappa = 0) and the constant
    scattering of the paper's run, sigma rho = 3.9e4 cm^2/g x 1.67e-24 g/cm^3
    x 1.496e13 cm = 9.74e-7 per unit length; c_hat = c = 1;
    dt = cfl / (3 c_hat / dx)."""
    half = 0.5 * N * dx
    n = (N, N, N)
    faces = [uniform_faces(N, -half, half) for _ in range(3)]
    xc = 0.5 * (faces[0][1:] + faces[0][:-1])
    r2 = xc[None, None, :] ** 2 + xc[None, :, None] ** 2 + xc[:, None, None] ** 2
    gamma = 5.0 / 3.0
    f = _zeros((N, N, N))
    f["E"][:] = (1.0 + 100.0 * np.exp(-r2 / 25.0)) ** 4
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.0 / (gamma - 1.0)
    sigma = 3.9e4 * 1.67e-24 * 1.496e13
    return Problem("p0", CARTESIAN, 3, n, faces, [[PERIODIC] * 2] * 3,
                   c_hat=1.0, c=1.0, gamma=gamma,
                   opacity=dict(kind=OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=sigma),
                   fields=f, dt=cfl / (3.0 / dx), steps=steps)


# ----------------------------------------------------------------------------
# MLP surrogate data (2 -> 64 -> 64 -> 2, tanh, linear 2 -> 2 shortcut)
# ----------------------------------------------------------------------------

MLP_IN, MLP_HID, MLP_OUT = 2, 64, 2
# parameter order in the flat float vector (row-major matrices, out x in)
MLP_LAYOUT = (("W1", (64, 2)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (2, 64)), ("b3", (2,)), ("Ws", (2, 2)))
MLP_NPARAM = sum(int(np.prod(s)) for _, s in MLP_LAYOUT)
# training schedule used by the benchmark and the tests (Adam, cosine decay)
MLP_TRAIN = dict(batch=4096, steps=600000, lr=7e-4, lr_final=7e-7)


def mlp_unflatten(theta):
    out, o = {}, 0
    for name, shp in MLP_LAYOUT:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k]).reshape(shp)
        o += k
    return out


def mlp_init(seed=7):
    """Seeded Glorot-uniform hidden weights; zero biases, zero output layer and
    zero shortcut (float32).  The trainer fits the shortcut to the table by
    least squares, so the network starts at that plane and the tanh layers
    learn only the residual."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shp in MLP_LAYOUT:
        if name in ("W1", "W2"):
            fan_out, fan_in = shp
            lim = math.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-lim, lim, shp).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shp))))
    return np.concatenate(parts).astype(np.float32)


def mlp_samples(n, seed):
    """Uniform (log10 rho, log10 T) table-coordinates over the table domain.

    Returned as float32 [n][2] in table coordinates (lr, lt), i.e. already
    including the lookup offsets.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lr = rng.uniform(TABLE_LR[0], TABLE_LR[1], n)
    lt = rng.uniform(TABLE_LT[0], TABLE_LT[1], n)
    return np.ascontiguousarray(np.stack([lr, lt], axis=1).astype(np.float32))


# ----------------------------------------------------------------------------
# test problems from the scheme's test section
# ----------------------------------------------------------------------------

def make_shock_tube(which, N=256, t_end=20.0, cfl=0.4):
    """Optically thin 1D Riemann problems on [-20, 20], outflow, c_hat = 1."""
    n = (N, 1, 1)
    faces = _cart_faces(n, -20.0, 20.0)
    faces[1] = np.array([0.0, 1.0])
    faces[2] = np.array([0.0, 1.0])
    x = 0.5 * (faces[0][1:] + faces[0][:-1])
    f = _zeros((1, 1, N))
    left = x < 0
    if which == 1:
        f["E"][:] = 1.0
        f["Fy"][..., left] = 0.5
    else:
        f["E"][..., left] = 0.1
        f["E"][..., ~left] = 1.0
        f["Fx"][..., left] = 0.1
        f["Fy"][..., ~left] = 1.0
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.5
    dx = 40.0 / N
    steps = int(math.ceil(t_end / (cfl * dx)))
    return Problem(f"tube{which}", CARTESIAN, 1, n, faces, [[OUTFLOW] * 2] * 3,
                   c_hat=1.0, c=1.0,
                   opacity=dict(kind=OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.0),
                   fields=f, dt=t_end / steps, steps=steps)


def make_beam(N=300, steps=None, cfl=0.4):
    """Oblique free-streaming beam in a 5 x 5 box, outflow boundaries."""
    n = (N, N, 1)
    faces = _cart_faces(n, 0.0, 5.0)
    faces[2] = np.array([0.0, 1.0])
    xc = 0.5 * (faces[0][1:] + faces[0][:-1])
    yc = 0.5 * (faces[1][1:] + faces[1][:-1])
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    f = _zeros((1, N, N))
    E = np.full((N, N), 1e4)
    inb = (X >= 0.5) & (X <= 0.6) & (Y >= 0.3) & (Y <= 0.44)
    E[inb] = 1e12
    f["E"][0] = E
    f["Fx"][0][inb] = 1e12 / math.sqrt(2.0)
    f["Fy"][0][inb] = 1e12 / math.sqrt(2.0)
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.5
    dx = 5.0 / N
    dt = cfl / (1.0 / dx + 1.0 / dx)
    if steps is None:
        steps = int(5.0 / dt)
    return Problem("beam", CARTESIAN, 2, n, faces, [[OUTFLOW] * 2] * 3,
                   c_hat=1.0, c=1.0,
                   opacity=dict(kind=OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.0),
                   fields=f, dt=dt, steps=steps)


def make_shadow(nx=140, ny=40, absorb_only=1, t_end=2.0, cfl=0.4, a_rad=1e-12):
    """Shadow test of Sect. 3.3 in code units (length in cm, c = c_hat = 1):
    a 1 x 0.3 box (x in [-0.5, 0.5], y in [0, 0.3]), a free-streaming beam
    injected at x = -0.5 (fixed ghost state, T_r / T = 6, F_x = E), outflow at
    x = 0.5 and y = 0.3, reflective at y = 0; a spheroid of density 1000 in a
    background of density 1, rho = 1 + 999 / (1 + e^D),
    D = 10 [(x / 0.1)^2 + (y / 0.06)^2 - 1]; T = 1 everywhere, F = v = 0;
    kappa_P = kappa_R = 0.1 rho T^-3.5 (Kramers).  The radiation constant is
    small (a = 1e-12) so that, as in the paper's physical units, the gas heat
    capacity dwarfs the radiation energy and T stays put."""
    n = (nx, ny, 1)
    faces = [uniform_faces(nx, -0.5, 0.5), uniform_faces(ny, 0.0, 0.3), np.array([0.0, 1.0])]
    xc = 0.5 * (faces[0][1:] + faces[0][:-1])
    yc = 0.5 * (faces[1][1:] + faces[1][:-1])
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    D = 10.0 * ((X / 0.1) ** 2 + (Y / 0.06) ** 2 - 1.0)
    rho = 1.0 + 999.0 / (1.0 + np.exp(D))
    f = _zeros((1, ny, nx))
    f["rho"][0] = rho
    f["E"][:] = a_rad
    gamma = 5.0 / 3.0
    f["Eg"][0] = rho * 1.0 / (gamma - 1)
    Eb = a_rad * 6.0 ** 4
    dt = cfl / (1.0 / (faces[0][1] - faces[0][0]) + 1.0 / (faces[1][1] - faces[1][0]))
    p = Problem("shadow", CARTESIAN, 2, n, faces, [[FIXED, OUTFLOW], [REFLECT, OUTFLOW], [PERIODIC, PERIODIC]],
                c_hat=1.0, c=1.0, a_rad=a_rad, gamma=gamma,
                opacity=dict(kind=OPAC_POWERLAW, k0=0.1, rho0=1.0, alpha=1.0, T0=1.0, beta=-3.5, sigma=0.0),
                fields=f, dt=dt, steps=int(round(t_end / dt)),
                bc_state=[[(Eb, Eb, 0.0, 0.0), None], [None, None], [None, None]], absorb_only=absorb_only)
    return p


def make_multigroup(m=8, n=(128, 128, 128), seed=6, dt=None, steps=20):
    """Multigroup workload: the c1 turbulent-box recipe (seeded fields, periodic
    unit box) with the radiation split into m groups by seeded random
    fractions (each group keeps f <= 0.5).  Group edges are log-spaced
    between 0.3 and 20 (h nu / k in the temperature unit), Planck opacities
    log-spaced from 0.1 to 30, Rosseland from 0.3 to 10, scattering 0.1."""
    N = n[0]
    p = make_turbulent_box(N, seed, 5.2083e-5 * 128 / N if dt is None else dt, steps, f"mg{m}")
    if tuple(n) != (N, N, N):
        raise ValueError("cubic boxes only")
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    w = rng.uniform(0.5, 1.5, m)
    w /= w.sum()
    for k in ("E", "Fx", "Fy", "Fz"):
        p.fields[k] = np.ascontiguousarray(np.stack([p.fields[k] * w[g] for g in range(m)]))
    p.groups = dict(edges=list(np.geomspace(0.3, 20.0, m - 1)) if m > 1 else [],
                    kP=list(np.geomspace(0.1, 30.0, m)), kR=list(np.geomspace(0.3, 10.0, m)))
    p.opacity = dict(kind=OPAC_CONSTANT, kP=0.0, kR=0.0, sigma=0.1)
    return p


def make_uniform(geometry, n, ndim, E=1.0, F=(0.0, 0.0, 0.0), bc=PERIODIC,
                 faces=None, kP=0.0, kR=0.0, sigma=0.0, c_hat=1.0):
    """Spatially uniform radiation field on any grid (well-balance checks)."""
    shape = (n[2], n[1], n[0])
    f = _zeros(shape)
    f["E"][:] = E
    f["Fx"][:], f["Fy"][:], f["Fz"][:] = F
    f["rho"][:] = 1.0
    f["Eg"][:] = 1.5
    if faces is None:
        faces = _cart_faces(n)
    return Problem("uniform", geometry, ndim, tuple(n), faces, [[bc] * 2] * 3,
                   c_hat=c_hat, c=c_hat,
                   opacity=dict(kind=OPAC_CONSTANT, kP=kP, kR=kR, sigma=sigma),
                   fields=f, dt=0.0, steps=1)


def make_random_state(geometry, n, ndim, seed, faces, bc, fmax=0.9, c_hat=1.0,
                      opacity=None, vmax=0.0):
    """Smooth-plus-noise random state for parity tests on small grids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n[2], n[1], n[0])
    E = np.exp(0.5 * rng.standard_normal(shape))
    Fx, Fy, Fz = _random_flux(rng, E, fmax, shape)
    rho = np.exp(0.5 * rng.standard_normal(shape))
    T = np.exp(0.2 * rng.standard_normal(shape))
    v = [vmax * rng.uniform(-1, 1, shape) for _ in range(3)]
    gamma = 5.0 / 3.0
    f = dict(E=E, Fx=Fx, Fy=Fy, Fz=Fz, rho=rho, mx=rho * v[0], my=rho * v[1], mz=rho * v[2],
             Eg=rho * T / (gamma - 1) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
    if opacity is None:
        opacity = dict(kind=OPAC_CONSTANT, kP=1.0, kR=2.0, sigma=0.5)
    return Problem(f"rand{seed}", geometry, ndim, tuple(n), faces, bc,
                   c_hat=c_hat, c=c_hat, gamma=gamma, opacity=opacity, fields=f,
                   dt=0.0, steps=1)


WORKLOADS = {"c0": make_c0, "c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4}
