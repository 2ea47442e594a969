"""The largest grids: 1024^3 = 2^30 cells in both forms (32-bit cell
indices near their limit, tens of GB of device state), one step, checked
cell by cell on a seeded sample against the oracle run on each sampled
cell's 5x5x5 neighbourhood (all that one step of the cell depends on:
slopes reach two cells, the implicit step is local), plus the conserved
totals of the whole grid.  The state is drawn on the device."""
import math

import numpy as np
import pytest
import torch

from paper_2606_26268_amd import inputs as I
from tests.gpu_common import TOL_P64, assert_close, assert_close_f32, fp32_response, say

pytestmark = pytest.mark.gpu

N = 1024
RADF = ("E", "Fx", "Fy", "Fz")
GASF = ("rho", "mx", "my", "mz", "Eg")


def _device_state(n, seed, dev):
    """Random radiation (|F| <= 0.6 E, isotropic directions), log-normal
    density, temperature in [1, 1.2], gas at rest; float64 on the device."""
    g = torch.Generator(device=dev).manual_seed(seed)
    shape = (n, n, n)

    def u():
        return torch.rand(shape, generator=g, device=dev, dtype=torch.float64)

    f = {"E": 1.0 + 0.5 * u()}
    a = 0.6 * u() * f["E"]
    mu = 2.0 * u() - 1.0
    ph = 2.0 * math.pi * u()
    st = torch.sqrt(1.0 - mu * mu)
    f["Fx"] = a * st * torch.cos(ph)
    f["Fy"] = a * st * torch.sin(ph)
    f["Fz"] = a * mu
    del a, mu, ph, st
    f["rho"] = torch.exp(0.3 * torch.randn(shape, generator=g, device=dev, dtype=torch.float64))
    f["Eg"] = f["rho"] * (1.0 + 0.2 * u()) * 1.5
    for k in ("mx", "my", "mz"):
        f[k] = torch.zeros(shape, device=dev, dtype=torch.float64)
    return f


def _problem(fields):
    faces = [I.uniform_faces(N, 0.0, 1.0) for _ in range(3)]
    p = I.Problem("max", I.CARTESIAN, 3, (N, N, N), faces, [[I.PERIODIC] * 2] * 3, c_hat=1.0, c=1.0,
                  opacity=dict(kind=I.OPAC_CONSTANT, kP=2.0, kR=1.0, sigma=0.5), fields=fields)
    p.dt = 0.4 / (3.0 * N)
    return p


def _samples(seed, count=48):
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (N - 1, N - 1, N - 1), (N - 1, 0, N // 2), (0, N - 1, 1), (N // 2, N - 2, N - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(count - len(pts))]
    return pts                                     # (i, j, k)


def _gather(t, pts, r):
    """Neighbourhoods (2r+1)^3 of each point with periodic wrap, as numpy."""
    out = []
    for i, j, k in pts:
        ii = [(i + d) % N for d in range(-r, r + 1)]
        jj = [(j + d) % N for d in range(-r, r + 1)]
        kk = [(k + d) % N for d in range(-r, r + 1)]
        blk = t[kk][:, jj][:, :, ii]
        out.append(blk.to("cpu", torch.float64).numpy())
    return out


@pytest.mark.parametrize("precision", ["f32", "p64"])
def test_max_size_step(orc, precision):
    from paper_2606_26268_amd import m1
    dev = torch.device("cuda:0")
    torch.cuda.empty_cache()
    say(f"case max size 1024^3 {precision}: drawing the state on the device")
    f = _device_state(N, 11, dev)
    p = _problem(f)
    s = m1.Solver(p, precision)
    p.fields = None                            # the solver holds the (converted) state
    del f
    torch.cuda.empty_cache()
    pts = _samples(5)
    # the solver's own inputs (FP32-rounded radiation in the FP32 form)
    nb = {k: _gather(s.t[k], pts, 2) for k in RADF + GASF}
    d0 = s.diagnostics()
    say("  one step")
    s.step(p.dt, 1)
    s.sync()
    d1 = s.diagnostics()
    got = {k: np.array([s.t[k][kk, jj, ii].item() for ii, jj, kk in pts]) for k in RADF + GASF}
    s.close()
    del s
    torch.cuda.empty_cache()
    # totals of the periodic box
    tot = abs(d1["total_energy"] - d0["total_energy"]) / d0["total_energy"]
    say(f"  total energy change {tot:.1e}, counters {d1['counters']}")
    assert tot <= (1e-6 if precision == "f32" else 1e-13)
    # each sampled cell against the oracle on its neighbourhood
    ref = {k: np.empty(len(pts)) for k in RADF + GASF}
    resp = {name: {k: np.empty(len(pts)) for k in RADF + GASF} for name in ("fp32", "flip")}
    for q in range(len(pts)):
        faces = [I.uniform_faces(5, 0.0, 5.0 / N) for _ in range(3)]
        loc = I.Problem("nb", I.CARTESIAN, 3, (5, 5, 5), faces, [[I.PERIODIC] * 2] * 3, c_hat=1.0, c=1.0,
                        opacity=p.opacity, fields={k: nb[k][q] for k in RADF + GASF})
        r, _ = orc.Oracle(loc).run(loc.fields, p.dt, 1)
        r32 = fp32_response(orc, loc, 1, dt=p.dt) if precision == "f32" else {"fp32": r, "flip": r}
        for k in RADF + GASF:
            ref[k][q] = r[k][2, 2, 2]
            for name in resp:
                resp[name][k][q] = r32[name][k][2, 2, 2]
    fields = ("E", "Fx", "Fy", "Fz", "mx", "my", "mz", "Eg")
    if precision == "p64":
        assert_close(got, ref, TOL_P64, fields=fields, label="max p64")
        return
    # FP32: the gas starts at rest, so after one step its momentum is only the
    # exchanged flux (dt c_hat rho chi ~ 2e-4 of F / c_hat), and the FP32
    # rounding of the stored F is large relative to it; the momentum is
    # judged against the flux scale F / c_hat it inherits that rounding from
    assert_close_f32(got, ref, resp, fields=("E", "Fx", "Fy", "Fz", "Eg"), label="max f32")
    for q, c in enumerate(("x", "y", "z")):
        err = np.abs(got["m" + c] - ref["m" + c]).sum() / (np.abs(ref["F" + c]).sum() / 1.0)
        say(f"  m{c}: sum |dm| / sum |F / c_hat| = {err:.1e}")
        assert err <= 1e-6, (c, err)


def test_cell_count_limit():
    """More than 2^31 - 2^16 cells is refused before anything is allocated."""
    from paper_2606_26268_amd import m1
    n = (65536, 32768, 1)
    faces = [I.uniform_faces(n[0], 0.0, 1.0), I.uniform_faces(n[1], 0.0, 1.0), np.array([0.0, 1.0])]
    with pytest.raises(m1.M1Error) as e:
        m1.m1_create(2, n, faces, [[I.PERIODIC] * 2] * 3, I.CARTESIAN, 1.0, m1.m1_params_default(1.0))
    assert e.value.status == m1.M1_EINVAL
