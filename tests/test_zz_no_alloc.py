"""m1_step_noalloc (the allocation-free step, through the C ABI) against the
allocating path on the same inputs: m1_bind_state followed by
m1_step_explicit and m1_step_implicit.  Two calls in a row on one device,
the second on a smaller grid (the static buffer keeps the first call's
contents), in both forms; then the size limit and the unsupported cases."""
import numpy as np
import pytest
import torch

from gpu_common import TOL_P64, assert_close, say

pytestmark = pytest.mark.gpu


def _problems():
    from paper_2606_26268_amd import inputs as I
    big = I.make_c3(nr=40, nth=24, nph=36, dt=2e-5)           # spherical, table opacity
    faces = [I.uniform_faces(20, 0.0, 1.0) for _ in range(3)]
    small = I.make_random_state(I.CARTESIAN, (20, 18, 16), 3, 9,
                                [faces[0], I.uniform_faces(18, 0.0, 1.0), I.uniform_faces(16, 0.0, 1.0)],
                                [[I.PERIODIC] * 2] * 3, fmax=0.8, c_hat=2.0)
    small.dt = 0.4 / (2.0 * 3 * 20)
    return big, small


@pytest.mark.parametrize("precision", ["p64", "f32"])
def test_noalloc_step_matches_the_bound_step(precision):
    from paper_2606_26268_amd import m1
    for prob in _problems():
        ref = m1.Solver(prob, precision)
        other = m1.Solver(prob, precision)
        before = {k: v.clone() for k, v in other.t.items()}
        # the caller's own arrays (copies of the same input)
        mine = {k: v.clone() for k, v in other.t.items()}
        torch.cuda.synchronize()
        say(f"  {precision} {prob.name} {prob.n}: m1_step_noalloc")
        m1.m1_step_noalloc(other.ctx, mine, prob.dt)
        ref.step(prob.dt)
        other.sync()
        a = ref.state()
        got = {k: v.detach().to("cpu", torch.float64).numpy().reshape(a[k].shape) for k, v in mine.items()}
        same = all(np.array_equal(got[k], a[k]) for k in a)
        say(f"    bitwise equal to the bound step: {same}")
        assert_close(got, a, TOL_P64, label=f"noalloc {precision} {prob.name}")
        # the context's own binding was not touched
        for k in before:
            assert torch.equal(other.t[k], before[k]), k
        ref.close()
        other.close()


def test_noalloc_limits():
    from paper_2606_26268_amd import inputs as I
    from paper_2606_26268_amd import m1
    # 3e6 cells in FP64 need 6 x 24 MB: more than the 128 MiB buffer
    n = (300, 100, 100)
    faces = [I.uniform_faces(k, 0.0, 1.0) for k in n]
    par = m1.m1_params_default(1.0)
    ctx = m1.m1_create(3, n, faces, [[I.PERIODIC] * 2] * 3, I.CARTESIAN, 1.0, par)
    t = {k: torch.zeros(256, dtype=torch.float64, device="cuda") for k in
         ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")}
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_noalloc(ctx, t, 1e-3)
    assert e.value.status == m1.M1_EINVAL and "static buffer" in str(e.value)
    m1.m1_destroy(ctx)
    # frequency groups are not supported
    p = I.make_multigroup(2, (8, 8, 8), steps=1)
    s = m1.Solver(p, "p64")
    with pytest.raises(m1.M1Error) as e:
        m1.m1_step_noalloc(s.ctx, s.t, p.dt)
    assert e.value.status == m1.M1_ENOTSUP
    s.close()
