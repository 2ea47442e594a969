"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  The C sources in
this folder share no code with the HIP path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["closure.c", "transport.c", "implicit.c", "mlp.c", "multigroup.c"]
LIB = os.path.join(HERE, "liboracle.so")

NCNT = 4
CNT_EFLOOR, CNT_FFIX_TRANSPORT, CNT_FFIX_IMPLICIT, CNT_FORM_MISMATCH = range(4)


def build(force=False):
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math, no FMA)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    hdr = os.path.join(HERE, "m1_oracle.h")
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(s) for s in srcs + [hdr, __file__])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", tmp] + srcs + ["-lm"]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


class Problem(C.Structure):
    _fields_ = [
        ("geometry", C.c_int), ("ndim", C.c_int),
        ("n", C.c_int * 3),
        ("faces", C.POINTER(C.c_double) * 3),
        ("bc", (C.c_int * 2) * 3),
        ("c_hat", C.c_double), ("c", C.c_double), ("a_rad", C.c_double),
        ("gamma", C.c_double), ("e_floor", C.c_double),
        ("opac_kind", C.c_int),
        ("kP", C.c_double), ("kR", C.c_double), ("sigma", C.c_double),
        ("pl_k0", C.c_double), ("pl_rho0", C.c_double), ("pl_alpha", C.c_double),
        ("pl_T0", C.c_double), ("pl_beta", C.c_double),
        ("tab_nr", C.c_int), ("tab_nt", C.c_int),
        ("tab_lr0", C.c_double), ("tab_lr1", C.c_double), ("tab_lt0", C.c_double),
        ("tab_lt1", C.c_double), ("tab_lr_off", C.c_double), ("tab_lt_off", C.c_double),
        ("tab_kP", C.POINTER(C.c_float)), ("tab_kR", C.POINTER(C.c_float)),
        ("mlp_theta", C.POINTER(C.c_double)),
        ("mlp_norm", C.c_double * 4),
        ("mlp_bf16", C.c_int),
        ("recon", C.c_int),
        ("riemann", C.c_int),
        ("bc_state", ((C.c_double * 4) * 2) * 3),
        ("irr", C.POINTER(C.c_double)),
        ("absorb_only", C.c_int),
        ("limiter", C.c_int),
        ("face_noise", C.c_double),
        ("noise_seed", C.c_ulonglong),
    ]


_dp = C.POINTER(C.c_double)
_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        L.m1o_xi.restype = C.c_double
        L.m1o_xi.argtypes = [C.c_double]
        L.m1o_eddington.argtypes = [C.c_double] * 4 + [_dp, _dp, _dp]
        L.m1o_speeds.argtypes = [C.c_double] * 4 + [C.c_int, _dp, _dp]
        L.m1o_flux.argtypes = [C.c_double] * 4 + [C.c_int, _dp]
        L.m1o_hll.argtypes = [_dp, _dp, C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
        L.m1o_vanleer.restype = C.c_double
        L.m1o_vanleer.argtypes = [C.c_double, C.c_double]
        L.m1o_limo3.restype = C.c_double
        L.m1o_limo3.argtypes = [C.c_double, C.c_double]
        L.m1o_ffix.restype = C.c_int
        L.m1o_ffix.argtypes = [_dp, _dp, C.c_double, _dp]
        L.m1o_face_fix.restype = C.c_int
        L.m1o_face_fix.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp]
        L.m1o_lf.argtypes = [_dp, _dp, C.c_int, C.c_double, C.c_double, _dp]
        L.m1o_cell_geometry.argtypes = [C.POINTER(Problem), C.c_int, C.c_int, C.c_int, _dp]
        L.m1o_max_dt.restype = C.c_double
        L.m1o_max_dt.argtypes = [C.POINTER(Problem), C.c_double]
        pp = C.POINTER(_dp)
        cnt = C.POINTER(C.c_longlong)
        L.m1o_explicit.argtypes = [C.POINTER(Problem), C.c_double, pp, pp, cnt]
        L.m1o_implicit.argtypes = [C.POINTER(Problem), C.c_double, pp, pp, cnt]
        L.m1o_run.argtypes = [C.POINTER(Problem), C.c_double, C.c_int, pp, cnt]
        L.m1o_run_rk2.argtypes = [C.POINTER(Problem), C.c_double, C.c_int, pp, cnt]
        L.m1o_implicit_cell.argtypes = [C.c_double] * 10 + [_dp]
        L.m1o_opacity.argtypes = [C.POINTER(Problem), C.c_double, C.c_double, _dp, _dp]
        L.m1o_opacity_many.argtypes = [C.POINTER(Problem), C.c_long, _dp, _dp, _dp, _dp]
        L.m1o_mlp_nparam.restype = C.c_int
        L.m1o_mlp_forward.argtypes = [_dp, C.c_int, C.c_long, _dp, _dp]
        L.m1o_mlp_loss_grad.restype = C.c_double
        L.m1o_mlp_loss_grad.argtypes = [_dp, C.c_int, C.c_long, _dp, _dp, _dp]
        L.m1o_adam.argtypes = [C.c_long, _dp, _dp, _dp, _dp, C.c_long] + [C.c_double] * 4
        L.m1o_planck_cdf.restype = C.c_double
        L.m1o_planck_cdf.argtypes = [C.c_double]
        L.m1o_group_fractions.argtypes = [C.c_int, _dp, C.c_double, _dp]
        L.m1o_mg_cell.restype = C.c_int
        L.m1o_mg_cell.argtypes = [C.c_int, _dp] + [C.c_double] * 2 + [_dp] + [C.c_double] * 5 + [_dp, C.c_double, _dp]
        L.m1o_run_mg.restype = C.c_int
        L.m1o_run_mg.argtypes = [C.POINTER(Problem), C.c_int, _dp, _dp, _dp, C.c_double, C.c_int, pp, pp, cnt]
        L.m1o_run_mg_rk2.restype = C.c_int
        L.m1o_run_mg_rk2.argtypes = [C.POINTER(Problem), C.c_int, _dp, _dp, _dp, C.c_double, C.c_int, pp, pp, cnt]
        L.m1o_bf16_round.restype = C.c_double
        L.m1o_bf16_round.argtypes = [C.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_dp)


class Oracle:
    """Holds an ``m1o_problem`` built from an ``inputs.Problem``-like object.

    ``mlp`` (optional): dict(theta=float64 vector, norm=(mP, sP, mR, sR),
    bf16=bool) used when the opacity kind is the MLP.
    """

    def __init__(self, prob, mlp=None):
        self.prob = prob
        self._keep = []
        P = Problem()
        P.geometry = prob.geometry
        P.ndim = prob.ndim
        for d in range(3):
            P.n[d] = int(prob.n[d])
            f = np.ascontiguousarray(prob.faces[d], dtype=np.float64)
            assert f.shape == (prob.n[d] + 1,)
            self._keep.append(f)
            P.faces[d] = _ptr(f)
            P.bc[d][0], P.bc[d][1] = prob.bc[d]
        P.c_hat, P.c, P.a_rad = prob.c_hat, prob.c, prob.a_rad
        P.gamma, P.e_floor = prob.gamma, prob.e_floor
        P.recon = getattr(prob, "recon", 0)
        P.riemann = getattr(prob, "riemann", 0)
        P.absorb_only = int(getattr(prob, "absorb_only", 0))
        P.limiter = int(getattr(prob, "limiter", 0))
        bs = getattr(prob, "bc_state", None)
        if bs is not None:
            for d in range(3):
                for side in range(2):
                    if bs[d][side] is not None:
                        for v in range(4):
                            P.bc_state[d][side][v] = float(bs[d][side][v])
        irr = getattr(prob, "irr", None)
        if irr is not None:
            q = np.ascontiguousarray(irr, dtype=np.float64).ravel()
            assert q.size == int(np.prod(prob.n))
            self._keep.append(q)
            P.irr = _ptr(q)
        op = prob.opacity
        P.opac_kind = op["kind"]
        P.sigma = op.get("sigma", 0.0)
        if op["kind"] == 0:
            P.kP, P.kR = op["kP"], op["kR"]
        elif op["kind"] == 1:
            P.pl_k0, P.pl_rho0, P.pl_alpha = op["k0"], op["rho0"], op["alpha"]
            P.pl_T0, P.pl_beta = op["T0"], op["beta"]
        if op["kind"] in (2, 3):
            P.tab_nr, P.tab_nt = op["nr"], op["nt"]
            P.tab_lr0, P.tab_lr1 = op["lr0"], op["lr1"]
            P.tab_lt0, P.tab_lt1 = op["lt0"], op["lt1"]
            P.tab_lr_off, P.tab_lt_off = op["lr_off"], op["lt_off"]
            kp = np.ascontiguousarray(op["log10_kP"], dtype=np.float32)
            kr = np.ascontiguousarray(op["log10_kR"], dtype=np.float32)
            self._keep += [kp, kr]
            P.tab_kP = kp.ctypes.data_as(C.POINTER(C.c_float))
            P.tab_kR = kr.ctypes.data_as(C.POINTER(C.c_float))
        if op["kind"] == 3:
            assert mlp is not None, "MLP opacity needs weights"
            th = np.ascontiguousarray(mlp["theta"], dtype=np.float64)
            self._keep.append(th)
            P.mlp_theta = _ptr(th)
            for i in range(4):
                P.mlp_norm[i] = float(mlp["norm"][i])
            P.mlp_bf16 = 1 if mlp.get("bf16", True) else 0
        self.P = P
        self.N = int(np.prod(prob.n))

    # -- helpers ------------------------------------------------------------
    def _arrs(self, fields, names):
        out = []
        for k in names:
            a = fields[k]
            assert a.dtype == np.float64 and a.flags.c_contiguous and a.size == self.N, k
            out.append(a)
        return out

    @staticmethod
    def _pp(arrs):
        return (_dp * len(arrs))(*[_ptr(a) for a in arrs])

    # -- steps --------------------------------------------------------------
    def run(self, fields, dt, nsteps, rk2=False):
        """Advance a copy of ``fields`` by nsteps (Euler split steps, or RK2
        with rk2=True); returns (fields, counters)."""
        st = {k: np.ascontiguousarray(v, dtype=np.float64).copy() for k, v in fields.items()}
        names = ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")
        arrs = self._arrs(st, names)
        cnt = (C.c_longlong * NCNT)()
        fn = lib().m1o_run_rk2 if rk2 else lib().m1o_run
        rc = fn(C.byref(self.P), dt, int(nsteps), self._pp(arrs), cnt)
        if rc != 0:
            raise MemoryError("oracle run failed")
        return st, np.array(list(cnt))

    def run_mg(self, fields, dt, nsteps, rk2=False):
        """Multigroup run (prob.groups = dict(edges, kP, kR)): fields E, Fx,
        Fy, Fz have a leading group axis; Euler split steps, or RK2 with
        rk2=True; returns (fields, counters)."""
        gr = self.prob.groups
        m = len(gr["kP"])
        edges = np.ascontiguousarray(gr["edges"], dtype=np.float64).reshape(-1)
        assert edges.size == m - 1
        kP = np.ascontiguousarray(gr["kP"], dtype=np.float64)
        kR = np.ascontiguousarray(gr["kR"], dtype=np.float64)
        st = {k: np.ascontiguousarray(v, dtype=np.float64).copy() for k, v in fields.items()}
        rad = []
        for g in range(m):
            for k in ("E", "Fx", "Fy", "Fz"):
                a = st[k][g]
                assert a.flags.c_contiguous and a.size == self.N
                rad.append(a)
        gas = self._arrs(st, ("rho", "mx", "my", "mz", "Eg"))
        cnt = (C.c_longlong * NCNT)()
        fn = lib().m1o_run_mg_rk2 if rk2 else lib().m1o_run_mg
        rc = fn(C.byref(self.P), m, _ptr(edges), _ptr(kP), _ptr(kR), dt, int(nsteps), self._pp(rad), self._pp(gas), cnt)
        if rc != 0:
            raise RuntimeError("oracle multigroup run failed")
        return st, np.array(list(cnt))

    def explicit(self, fields, dt):
        names = ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")
        st = {k: np.ascontiguousarray(fields[k], dtype=np.float64) for k in names}
        arrs = self._arrs(st, names)
        out = [np.empty(self.N) for _ in range(4)]
        cnt = (C.c_longlong * NCNT)()
        rc = lib().m1o_explicit(C.byref(self.P), dt, self._pp(arrs), self._pp(out), cnt)
        if rc != 0:
            raise MemoryError("oracle explicit failed")
        shp = fields["E"].shape
        return {k: o.reshape(shp) for k, o in zip(("E", "Fx", "Fy", "Fz"), out)}, np.array(list(cnt))

    def implicit(self, fields, star, dt):
        names = ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg")
        st = {k: np.ascontiguousarray(fields[k], dtype=np.float64).copy() for k in names}
        arrs = self._arrs(st, names)
        sa = [np.ascontiguousarray(star[k], dtype=np.float64) for k in ("E", "Fx", "Fy", "Fz")]
        cnt = (C.c_longlong * NCNT)()
        lib().m1o_implicit(C.byref(self.P), dt, self._pp(sa), self._pp(arrs), cnt)
        return st, np.array(list(cnt))

    def max_dt(self, cfl):
        return lib().m1o_max_dt(C.byref(self.P), cfl)

    def cell_geometry(self, i, j, k):
        out = np.zeros(12)
        lib().m1o_cell_geometry(C.byref(self.P), i, j, k, _ptr(out))
        return out

    def volumes(self):
        n = self.prob.n
        V = np.empty((n[2], n[1], n[0]))
        for k in range(n[2]):
            for j in range(n[1]):
                for i in range(n[0]):
                    V[k, j, i] = self.cell_geometry(i, j, k)[0]
        return V

    def opacity(self, rho, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        kP, kR = np.empty_like(rho), np.empty_like(rho)
        lib().m1o_opacity_many(C.byref(self.P), rho.size, _ptr(rho), _ptr(T), _ptr(kP), _ptr(kR))
        return kP, kR


# -- pointwise functions ------------------------------------------------------

def xi(f):
    return lib().m1o_xi(float(f))


def eddington(E, F):
    f, x = C.c_double(), C.c_double()
    D = np.zeros(9)
    lib().m1o_eddington(float(E), float(F[0]), float(F[1]), float(F[2]), C.byref(f), C.byref(x), _ptr(D))
    return f.value, x.value, D.reshape(3, 3)


def speeds(E, F, d):
    a, b = C.c_double(), C.c_double()
    lib().m1o_speeds(float(E), float(F[0]), float(F[1]), float(F[2]), int(d), C.byref(a), C.byref(b))
    return a.value, b.value


def flux(E, F, d):
    out = np.zeros(4)
    lib().m1o_flux(float(E), float(F[0]), float(F[1]), float(F[2]), int(d), _ptr(out))
    return out


def hll(UL, UR, d, tau=0.0, c_hat=1.0):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    out = np.zeros(4)
    SL, SR = C.c_double(), C.c_double()
    lib().m1o_hll(_ptr(UL), _ptr(UR), int(d), float(tau), float(c_hat), _ptr(out), C.byref(SL), C.byref(SR))
    return out, SL.value, SR.value


def vanleer(dl, dr):
    return lib().m1o_vanleer(float(dl), float(dr))


def limo3(dfar, dnear):
    return lib().m1o_limo3(float(dfar), float(dnear))


def ffix(Ef, Ff, Ec, Fc):
    e = C.c_double(Ef)
    Ff = np.ascontiguousarray(Ff, dtype=np.float64).copy()
    Fc = np.ascontiguousarray(Fc, dtype=np.float64)
    br = lib().m1o_ffix(C.byref(e), _ptr(Ff), float(Ec), _ptr(Fc))
    return br, e.value, Ff


def face_fix(recon, Ef, Ff, Ec, Fc):
    e = C.c_double(Ef)
    Ff = np.ascontiguousarray(Ff, dtype=np.float64).copy()
    Fc = np.ascontiguousarray(Fc, dtype=np.float64)
    br = lib().m1o_face_fix(int(recon), C.byref(e), _ptr(Ff), float(Ec), _ptr(Fc))
    return br, e.value, Ff


def lf(UL, UR, d, tau=0.0, c_hat=1.0):
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    out = np.zeros(4)
    lib().m1o_lf(_ptr(UL), _ptr(UR), int(d), float(tau), float(c_hat), _ptr(out))
    return out


def implicit_cell(Es, Cv, T, kP, rho, dt, c_hat, c, a=1.0, S=0.0):
    """Single-cell implicit solve; S = irradiation energy deposited in the
    step (added to the S_1 row)."""
    out = np.zeros(4)
    lib().m1o_implicit_cell(float(Es), float(Cv), float(T), float(kP), float(rho), float(dt),
                            float(c_hat), float(c), float(a), float(S), _ptr(out))
    return out


def mlp_nparam():
    return lib().m1o_mlp_nparam()


def mlp_forward(theta, x, bf16=False):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    y = np.empty_like(x)
    lib().m1o_mlp_forward(_ptr(theta), int(bf16), x.shape[0], _ptr(x), _ptr(y))
    return y


def mlp_loss_grad(theta, x, t, bf16=False):
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 2)
    t = np.ascontiguousarray(t, dtype=np.float64).reshape(-1, 2)
    g = np.zeros_like(theta)
    loss = lib().m1o_mlp_loss_grad(_ptr(theta), int(bf16), x.shape[0], _ptr(x), _ptr(t), _ptr(g))
    return loss, g


def adam(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().m1o_adam(theta.size, _ptr(theta), _ptr(g), _ptr(m), _ptr(v), int(step), lr, b1, b2, eps)


def bf16_round(x):
    return lib().m1o_bf16_round(float(x))


def planck_cdf(x):
    return lib().m1o_planck_cdf(float(x))


def group_fractions(edges, T):
    edges = np.ascontiguousarray(edges, dtype=np.float64).reshape(-1)
    b = np.zeros(edges.size + 1)
    lib().m1o_group_fractions(edges.size + 1, _ptr(edges), float(T), _ptr(b))
    return b


def mg_cell(Es, Cv, T, kP, rho, dt, c_hat, c, a, b, S=0.0):
    Es = np.ascontiguousarray(Es, dtype=np.float64)
    kP = np.ascontiguousarray(kP, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.zeros(Es.size + 1)
    rc = lib().m1o_mg_cell(Es.size, _ptr(Es), float(Cv), float(T), _ptr(kP), float(rho), float(dt),
                           float(c_hat), float(c), float(a), _ptr(b), float(S), _ptr(out))
    if rc != 0:
        raise RuntimeError("singular multigroup system")
    return out


def set_threads(n):
    """Number of OpenMP threads the oracle's parallel loops use from now on
    (results do not depend on it: cells are independent, sums are serial)."""
    lib().omp_set_num_threads.argtypes = [C.c_int]
    lib().omp_set_num_threads(int(n))


def max_threads():
    lib().omp_get_max_threads.restype = C.c_int
    return int(lib().omp_get_max_threads())
