"""The seeded workloads have the sizes and statistics their definitions state."""
import numpy as np

from paper_2606_26268_amd import inputs as I


def test_grf_unit_variance_and_spectrum():
    rng = np.random.Generator(np.random.PCG64(0))
    w = rng.standard_normal((32, 32, 32))
    g = I.grf_from_white(w, -1.0)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1) < 1e-12
    # power in shells falls as k^-2 (times the k^2 shell area -> flat per shell)
    P = np.abs(np.fft.fftn(g)) ** 2
    k = I._kmag(g.shape)
    lo = P[(k > 2) & (k < 3)].mean()
    hi = P[(k > 8) & (k < 9)].mean()
    assert 0.5 < (lo / hi) / (8.5 / 2.5) ** 2 < 2.0


def test_turbulent_box_statistics():
    p = I.make_turbulent_box(32, 1, 1e-4, 1, "t")
    f = p.fields
    assert p.shape == (32, 32, 32) and p.ncells == 32 ** 3
    lnr = np.log(f["rho"])
    assert abs(lnr.std() - 1.0) < 1e-12 and abs(lnr.mean() + 0.5) < 1e-12
    T = (f["Eg"] - 0.5 * (f["mx"] ** 2 + f["my"] ** 2 + f["mz"] ** 2) / f["rho"]) / (f["rho"] / (p.gamma - 1))
    assert abs(np.abs(T - 1).max() - 0.3) < 1e-12
    v2 = (f["mx"] ** 2 + f["my"] ** 2 + f["mz"] ** 2) / f["rho"] ** 2
    assert abs(np.sqrt(v2.mean()) - 0.5) < 1e-12
    np.testing.assert_allclose(f["E"], T ** 4, rtol=1e-12)
    Fn = np.sqrt(f["Fx"] ** 2 + f["Fy"] ** 2 + f["Fz"] ** 2)
    assert (Fn <= 0.5 * f["E"]).all() and (Fn / f["E"]).max() > 0.49


def test_c0_c3_shapes_and_ranges():
    p = I.make_c0()
    assert p.n == (256, 1, 1) and p.steps == 100 and p.dt == 1.5625e-4
    p = I.make_c3(nr=24, nth=12, nph=24)
    f = p.fields
    assert p.shape == (24, 12, 24)
    assert abs(p.faces[0][0] - 1) < 1e-15 and abs(p.faces[0][-1] - 100) < 1e-12
    assert abs(p.faces[1][-1] - np.pi) < 1e-15 and abs(p.faces[2][-1] - 2 * np.pi) < 1e-15
    lr = np.log10(f["rho"]) + p.opacity["lr_off"]
    T = f["Eg"] / (f["rho"] / (p.gamma - 1))
    lt = np.log10(T) + p.opacity["lt_off"]
    assert lr.min() > -12 and lr.max() < 0 and lt.min() >= 3 - 1e-9 and lt.max() <= 4 + 1e-9


def test_table_and_samples():
    t = I.make_table()
    assert t["log10_kP"].shape == (128, 128) and t["log10_kP"].dtype == np.float32
    s = I.mlp_samples(1000, 4)
    assert s.shape == (1000, 2) and s.dtype == np.float32
    assert s[:, 0].min() >= -12 and s[:, 0].max() <= 0 and s[:, 1].min() >= 2 and s[:, 1].max() <= 6
    assert not np.array_equal(I.mlp_samples(10, 4), I.mlp_samples(10, 5))
    np.testing.assert_array_equal(I.mlp_samples(10, 4), I.mlp_samples(10, 4))
