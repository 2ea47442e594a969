"""Argument validation of the C ABI, on the host (no GPU): every call that
receives an invalid argument returns M1_EINVAL with a message naming the
problem, before any device call, and leaves its output untouched (m1_create
returns a null context).  m1_params_default is checked in test_abi."""
import math
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_26268_amd", "libm1.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="HIP library not built")


def _grid(m1, ndim=3, n=(4, 4, 4), faces=None, bc=None):
    g = m1.m1_grid()
    g.ndim = ndim
    keep = []
    for d in range(3):
        g.n[d] = n[d]
        f = np.ascontiguousarray(faces[d] if faces else np.arange(n[d] + 1, dtype=np.float64))
        keep.append(f)
        g.faces[d] = f.ctypes.data_as(m1.C.POINTER(m1.C.c_double))
        b = bc[d] if bc else (1, 1)
        g.bc[d][0], g.bc[d][1] = b
    return g, keep


def _create(m1, g, geom=0, c_hat=1.0, params=None):
    ctx = m1.C.c_void_p(12345)
    st = m1.lib().m1_create(m1.C.byref(g), geom, c_hat, m1.C.byref(params) if params is not None else None,
                            m1.C.byref(ctx))
    return st, ctx.value, m1.m1_last_error()


CASES = [
    ("ndim 0", dict(ndim=0), "ndim"),
    ("ndim 4", dict(ndim=4), "ndim"),
    ("geometry", dict(geom=3), "geometry"),
    ("c_hat zero", dict(c_hat=0.0), "c_hat"),
    ("c_hat nan", dict(c_hat=math.nan), "c_hat"),
    ("c_hat inf", dict(c_hat=math.inf), "c_hat"),
    ("no cells", dict(n=(0, 4, 4)), "n[d]"),
    ("inactive direction with cells", dict(ndim=2, n=(4, 4, 2)), "inactive"),
    ("boundary code", dict(bc=((1, 1), (1, 7), (1, 1))), "boundary"),
    ("unpaired periodic", dict(bc=((0, 1), (1, 1), (1, 1))), "paired"),
    ("reflective single cell", dict(ndim=2, n=(4, 1, 1), bc=((1, 1), (2, 1), (1, 1))), "reflective"),
    ("faces not increasing", dict(faces=[np.array([0, 1, 1, 2, 3.0]), np.arange(5.0), np.arange(5.0)]), "increasing"),
    ("faces nan", dict(faces=[np.array([0, 1, math.nan, 2, 3.0]), np.arange(5.0), np.arange(5.0)]), "increasing"),
    ("negative radius", dict(geom=2, faces=[np.linspace(-1, 1, 5), np.linspace(0, 3, 5), np.linspace(0, 6, 5)]),
     "radius"),
    ("theta past pi", dict(geom=2, faces=[np.linspace(1, 2, 5), np.linspace(0, 3.5, 5), np.linspace(0, 6, 5)]),
     "theta"),
]


@pytest.mark.parametrize("name,kw,word", CASES, ids=[c[0] for c in CASES])
def test_create_rejects(name, kw, word):
    from paper_2606_26268_amd import m1
    geom = kw.pop("geom", 0)
    c_hat = kw.pop("c_hat", 1.0)
    g, keep = _grid(m1, **kw)
    st, ctx, msg = _create(m1, g, geom, c_hat)
    assert st == m1.M1_EINVAL and ctx is None and word in msg, (st, ctx, msg)


def test_create_rejects_too_many_cells():
    from paper_2606_26268_amd import m1
    n = (2048, 1024, 1024)                         # 2^31 cells
    faces = [np.arange(k + 1, dtype=np.float64) for k in n]
    g, keep = _grid(m1, n=n, faces=faces)
    st, ctx, msg = _create(m1, g)
    assert st == m1.M1_EINVAL and ctx is None and "too many cells" in msg


PARAM_CASES = [("precision", 7, "precision"), ("recon", 3, "reconstruction"), ("riemann", 2, "Riemann"),
               ("absorb_only", 2, "absorb_only"), ("second_order", -1, "second_order"), ("limiter", 2, "limiter"), ("stream_reads", 3, "stream_reads"),
               ("c", 0.0, "gamma"), ("gamma", 1.0, "gamma"), ("a_rad", -1.0, "gamma")]


@pytest.mark.parametrize("field,value,word", PARAM_CASES, ids=[c[0] for c in PARAM_CASES])
def test_create_rejects_params(field, value, word):
    from paper_2606_26268_amd import m1
    p = m1.m1_params_default(1.0)
    setattr(p, field, value)
    g, keep = _grid(m1)
    st, ctx, msg = _create(m1, g, params=p)
    assert st == m1.M1_EINVAL and ctx is None and word in msg, (st, ctx, msg)


def test_null_arguments():
    from paper_2606_26268_amd import m1
    L, C = m1.lib(), m1.C
    g, keep = _grid(m1)
    ctx = C.c_void_p()
    assert L.m1_create(None, 0, 1.0, None, C.byref(ctx)) == m1.M1_EINVAL
    assert L.m1_create(C.byref(g), 0, 1.0, None, None) == m1.M1_EINVAL
    assert L.m1_params_default(1.0, None) == m1.M1_EINVAL
    for name, args in (("m1_set_stream", (None, None)), ("m1_bind_state", (None, None)),
                       ("m1_set_opacity_model", (None, 0, None)),
                       ("m1_set_opacity_mlp", (None, None, None)),
                       ("m1_max_dt", (None, 0.4, None)), ("m1_set_groups", (None, 1, None, None, None, 0.0)),
                       ("m1_set_boundary_state", (None, 0, 0, None))):
        st = getattr(L, name)(*args)
        assert st == m1.M1_EINVAL, (name, st)
        assert name.split("m1_", 1)[1].split("_")[0] in m1.m1_last_error() or "NULL" in m1.m1_last_error()
