"""The LimO3 reconstruction (Sect. 2.5, after Cada and Torrilhon 2009) on the
GPU against the oracle, through the C ABI: every geometry in one to three
dimensions with ragged tiles, the general 3D kernel with the other face
treatments, the Riemann solvers and reflective walls, the second-order
step, the two Sect. 3.1 shock tubes run to t = 20, and the 192x96x192
spherical grid in the launch configuration of the benchmark's forms."""
import numpy as np
import pytest

from paper_2606_26268_amd import inputs as I
from tests.gpu_common import TOL_P64, TOL_P64_F1, assert_close, assert_close_f32, fp32_response, run_gpu, say
from tests.test_gpu_parity import CASES, _problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("geom,n,ndim", CASES)
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_limo3_small_grids_all_geometries(orc, geom, n, ndim, precision):
    say(f"case limo3 geom={geom} n={n} ndim={ndim} {precision}")
    p = _problem(geom, n, ndim, seed=300 + 10 * geom + ndim)
    p.limiter = 1
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, cnt = o.run(p.fields, dt, 10)
    got, diag = run_gpu(p, precision, 10, dt=dt)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="limo3 p64")
        assert diag["counters"][:3] == list(cnt[:3])
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 10, dt=dt), label="limo3 f32")


@pytest.mark.parametrize("recon,riemann", [(0, 1), (1, 0), (2, 1)])
@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_limo3_general_kernel_variants(orc, recon, riemann, precision):
    """3D Cartesian box with reflective walls in x, LimO3 with each face
    treatment and both Riemann solvers (the general tiled kernel)."""
    say(f"case limo3 general recon={recon} riemann={riemann} {precision}")
    p = _problem(I.CARTESIAN, (37, 23, 19), 3, seed=41)
    p.bc = [[I.REFLECT, I.REFLECT], [I.OUTFLOW, I.OUTFLOW], [I.PERIODIC, I.PERIODIC]]
    p.limiter, p.recon, p.riemann = 1, recon, riemann
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, _ = o.run(p.fields, dt, 8)
    got, _ = run_gpu(p, precision, 8, dt=dt)
    if precision == "p64":
        # the PLUTO and clip treatments put faces at f = 1 exactly
        assert_close(got, ref, TOL_P64 if recon == 0 else TOL_P64_F1, label="limo3 general p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 8, dt=dt), label="limo3 general f32", f1=recon == 2)


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_limo3_second_order_step_spherical(orc, precision):
    from paper_2606_26268_amd import m1
    p = _problem(I.SPHERICAL, (24, 12, 22), 3, seed=43)
    p.limiter = 1
    o = orc.Oracle(p)
    dt = o.max_dt(0.4)
    ref, _ = o.run(p.fields, dt, 4, rk2=True)
    s = m1.Solver(p, precision, second_order=True)
    s.step(dt, 4, rk2=True)
    got = s.state()
    s.close()
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="limo3 rk2 p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 4, dt=dt, rk2=True), label="limo3 rk2 f32")


@pytest.mark.parametrize("which", [1, 2])
def test_limo3_shock_tubes(orc, which):
    """The Sect. 3.1 tubes at 2^8 cells, second-order steps to t = 20, FP64.
    The second tube is at f = 1 on both sides, where the signal speeds are
    square-root sensitive to rounding."""
    from paper_2606_26268_amd import m1
    p = I.make_shock_tube(which, N=256)
    p.limiter = 1
    say(f"case limo3 shock tube {which}, {p.steps} second-order steps")
    ref, cnt = orc.Oracle(p).run(p.fields, p.dt, p.steps, rk2=True)
    s = m1.Solver(p, "p64", second_order=True)
    s.step(p.dt, p.steps, rk2=True)
    got = s.state()
    s.close()
    assert_close(got, ref, TOL_P64 if which == 1 else TOL_P64_F1, fields=("E", "Fx", "Fy"),
                 label=f"limo3 tube {which}")


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_limo3_spherical_full_size_steps(orc, precision):
    """The 192x96x192 spherical grid with the table, three steps, LimO3."""
    p = I.make_c3()
    p.limiter = 1
    say(f"case limo3 spherical 192x96x192 {precision}, 3 steps")
    ref, _ = orc.Oracle(p).run(p.fields, p.dt, 3)
    got, _ = run_gpu(p, precision, 3)
    if precision == "p64":
        assert_close(got, ref, TOL_P64, label="limo3 c3 p64")
    else:
        assert_close_f32(got, ref, fp32_response(orc, p, 3), label="limo3 c3 f32")
