"""The library's time step (m1_max_dt, through the C ABI) against the
oracle's (m1o_max_dt, pinned to hand-worked values on the CPU) on grids of
every geometry in one to three dimensions, uniform and stretched: they
agree to one unit in the last place."""
import math

import numpy as np
import pytest

from gpu_common import say
from paper_2606_26268_amd import inputs as I

pytestmark = pytest.mark.gpu


def _grids():
    rng = np.random.default_rng(5)

    def stretched(n, lo, hi):
        w = rng.uniform(0.5, 1.5, n)
        return lo + (hi - lo) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])

    one = np.array([0.0, 1.0])
    out = []
    out.append(("cartesian 1D 256", I.CARTESIAN, 1, (256, 1, 1), [I.uniform_faces(256, 0, 1), one, one], 10.0))
    out.append(("cartesian 3D 128^3", I.CARTESIAN, 3, (128, 128, 128), [I.uniform_faces(128, 0, 1)] * 3, 20.0))
    out.append(("cartesian 2D stretched", I.CARTESIAN, 2, (37, 23, 1),
                [stretched(37, -1, 2), stretched(23, 0, 3), one], 3.0))
    out.append(("cylindrical 1D", I.CYLINDRICAL, 1, (40, 1, 1),
                [stretched(40, 0.5, 4.0), np.array([0.0, 2 * math.pi]), one], 1.0))
    out.append(("cylindrical 2D", I.CYLINDRICAL, 2, (31, 17, 1),
                [stretched(31, 0.0, 2.0), stretched(17, 0.0, 2 * math.pi), one], 2.0))
    out.append(("cylindrical 3D", I.CYLINDRICAL, 3, (12, 19, 9),
                [stretched(12, 0.1, 1.0), stretched(19, 0.0, 1.0), stretched(9, -1, 1)], 7.0))
    out.append(("spherical 1D", I.SPHERICAL, 1, (50, 1, 1),
                [np.geomspace(1, 10, 51), np.array([0.0, math.pi]), np.array([0.0, 2 * math.pi])], 1.0))
    out.append(("spherical 2D", I.SPHERICAL, 2, (24, 30, 1),
                [stretched(24, 0.2, 3.0), I.uniform_faces(30, 0.0, math.pi), np.array([0.0, 2 * math.pi])], 5.0))
    out.append(("spherical 3D stretched", I.SPHERICAL, 3, (14, 11, 13),
                [stretched(14, 1.0, 2.0), stretched(11, 0.2, 2.9), stretched(13, 0.0, 2.0)], 3.0))
    out.append(("spherical 192x96x192", I.SPHERICAL, 3, (192, 96, 192), I.spherical_faces(192, 96, 192), 20.0))
    return out


@pytest.mark.parametrize("case", _grids(), ids=lambda c: c[0])
def test_max_dt_matches_the_oracle(orc, case):
    from paper_2606_26268_amd import m1
    name, geom, ndim, n, faces, c_hat = case
    p = I.make_uniform(geom, n, ndim, faces=faces, bc=I.OUTFLOW, c_hat=c_hat)
    ref = orc.Oracle(p).max_dt(0.4)
    ctx = m1.m1_create(ndim, n, faces, [[I.OUTFLOW] * 2] * 3, geom, c_hat)
    try:
        got = m1.m1_max_dt(ctx, 0.4)
    finally:
        m1.m1_destroy(ctx)
    say(f"  {name}: library {got!r} oracle {ref!r}")
    assert abs(got - ref) <= np.spacing(ref), (got, ref)
