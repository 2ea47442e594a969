"""Pins of the oracle's MLP surrogate: forward pass against hand-built
networks with closed-form outputs, back-propagation against central finite
differences, bfloat16 rounding against a library conversion and the first
Adam step against its closed form."""
import math

import numpy as np
import pytest
import torch

from paper_2606_26268_amd import inputs as I


def _offsets():
    out, o = {}, 0
    for name, shp in I.MLP_LAYOUT:
        out[name] = (o, shp)
        o += int(np.prod(shp))
    return out


def test_parameter_count(orc):
    assert orc.mlp_nparam() == I.MLP_NPARAM == 4486


def test_forward_closed_form_network(orc):
    """Route x0 through hidden unit 3 of layer 1 and unit 5 of layer 2 to
    output 0: y0 = tanh(b * tanh(a * x0)); output 1 = shortcut only."""
    off = _offsets()
    th = np.zeros(I.MLP_NPARAM)
    a, b = 1.7, -0.8
    o, _ = off["W1"]; th[o + 3 * 2 + 0] = a          # W1[3][0]
    o, _ = off["W2"]; th[o + 5 * 64 + 3] = b         # W2[5][3]
    o, _ = off["W3"]; th[o + 0 * 64 + 5] = 1.0       # W3[0][5]
    o, _ = off["b3"]; th[o + 1] = 0.25               # b3[1]
    o, _ = off["Ws"]; th[o + 1 * 2 + 1] = -2.0       # Ws[1][1]
    x = np.array([[0.3, -0.4], [-0.9, 0.7], [0.0, 1.0]])
    y = orc.mlp_forward(th, x)
    for (x0, x1), (y0, y1) in zip(x, y):
        assert abs(y0 - math.tanh(b * math.tanh(a * x0))) < 1e-15
        assert abs(y1 - (0.25 - 2.0 * x1)) < 1e-15


def test_backprop_matches_finite_differences(orc):
    rng = np.random.default_rng(0)
    th = I.mlp_init(3).astype(np.float64) + 0.05 * rng.normal(size=I.MLP_NPARAM)
    x = rng.uniform(-1, 1, (32, 2))
    t = rng.normal(size=(32, 2))
    loss, g = orc.mlp_loss_grad(th, x, t)
    idx = rng.choice(I.MLP_NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [0, 127, 128, 191, 192, 4287, 4288, 4415, 4416, 4417, 4418, 4485]])
    for i in idx:
        h = 1e-5 * max(1.0, abs(th[i]))
        tp = th.copy(); tp[i] += h
        tm = th.copy(); tm[i] -= h
        fd = (orc.mlp_loss_grad(tp, x, t)[0] - orc.mlp_loss_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(fd), 1e-3), (i, fd, g[i])


def test_bf16_rounding_matches_library(orc):
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-6, 6, 2000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.tensor(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.bf16_round(a) for a in v])
    np.testing.assert_array_equal(got, ref)


def test_bf16_split_forward_close_to_exact(orc):
    rng = np.random.default_rng(2)
    th = I.mlp_init(5).astype(np.float64) + 0.05 * rng.normal(size=I.MLP_NPARAM)
    x = rng.uniform(-1, 1, (500, 2))
    y64 = orc.mlp_forward(th, x, bf16=False)
    y16 = orc.mlp_forward(th, x, bf16=True)
    # hi*hi + hi*lo + lo*hi keeps ~16 significant bits per product
    assert np.abs(y64 - y16).max() < 1e-4
    assert np.abs(y64 - y16).max() > 0


def test_adam_first_step_closed_form(orc):
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50); v = np.zeros(50)
    t0 = th.copy()
    orc.adam(th, g, m, v, 1, 1e-3, 0.9, 0.999, 1e-8)
    # bias-corrected first moments equal g and sqrt(g^2): step = -lr g/(|g|+eps)
    np.testing.assert_allclose(th - t0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_minimises_quadratic(orc):
    th = np.array([3.0, -2.0])
    m = np.zeros(2); v = np.zeros(2)
    for s in range(1, 3001):
        orc.adam(th, 2 * th, m, v, s, 1e-2)
    assert np.abs(th).max() < 1e-3
