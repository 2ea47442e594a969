"""Python binding of the C ABI in ``include/m1.h`` (``libm1.so``).

Each ``m1_*`` function here marshals arguments to the C call of the same
name; every step of the method runs in the library's HIP kernels.  PyTorch
only provides device memory and streams.  Importing this module fails loudly
if the HIP library has not been built.

``Solver`` is a convenience wrapper that owns torch tensors for one
synthetic ``inputs.Problem`` and drives the calls.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library then shares)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libm1.so")

M1_OK, M1_EINVAL, M1_ENOMEM, M1_EDEVICE, M1_ESTATE, M1_ENOTSUP = 0, -1, -2, -3, -4, -5
M1_CARTESIAN, M1_CYLINDRICAL, M1_SPHERICAL = 0, 1, 2
M1_BC_PERIODIC, M1_BC_OUTFLOW = 0, 1
M1_P64, M1_F32 = 0, 1
M1_OPAC_CONSTANT, M1_OPAC_POWERLAW = 0, 1
M1_RECON_FPRESERVE, M1_RECON_PLUTO, M1_RECON_CLIP = 0, 1, 2
M1_RIEMANN_HLL, M1_RIEMANN_LF = 0, 1
M1_LIMITER_PLM, M1_LIMITER_LIMO3 = 0, 1
M1_STREAM_AUTO, M1_STREAM_ON, M1_STREAM_OFF = 0, 1, 2
M1_MLP_NPARAM = 4486


class M1Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"m1 status {status}: {msg}")
        self.status = status


class m1_grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("faces", C.POINTER(C.c_double) * 3),
                ("bc", (C.c_int * 2) * 3)]


class m1_params(C.Structure):
    _fields_ = [("c", C.c_double), ("a_rad", C.c_double), ("gamma", C.c_double),
                ("precision", C.c_int), ("e_floor", C.c_double), ("recon", C.c_int), ("riemann", C.c_int),
                ("absorb_only", C.c_int),
                ("second_order", C.c_int), ("limiter", C.c_int), ("stream_reads", C.c_int)]


class m1_fields(C.Structure):
    _fields_ = [("E", C.c_void_p), ("Fx", C.c_void_p), ("Fy", C.c_void_p), ("Fz", C.c_void_p),
                ("rho", C.c_void_p), ("mx", C.c_void_p), ("my", C.c_void_p), ("mz", C.c_void_p),
                ("Eg", C.c_void_p)]


class m1_diag(C.Structure):
    _fields_ = [("rad_energy", C.c_double), ("total_energy", C.c_double), ("momentum", C.c_double * 3),
                ("min_E", C.c_double), ("max_f", C.c_double), ("counters", C.c_longlong * 4)]


class m1_mlp(C.Structure):
    _fields_ = [("theta", C.POINTER(C.c_float)), ("norm", C.c_double * 4)]


class m1_train_cfg(C.Structure):
    _fields_ = [("samples", C.c_void_p), ("n_train", C.c_long), ("n_eval", C.c_long),
                ("theta_init", C.POINTER(C.c_float)), ("batch", C.c_int), ("steps", C.c_long),
                ("lr", C.c_double), ("lr_final", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("keep_init", C.c_int)]


class m1_train_report(C.Structure):
    _fields_ = [("final_loss", C.c_double), ("max_rel_err_P", C.c_double),
                ("max_rel_err_R", C.c_double), ("seconds", C.c_double)]


# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = ("m1_params_default", "m1_create", "m1_destroy", "m1_set_stream", "m1_bind_state",
           "m1_set_opacity_model", "m1_set_opacity_table", "m1_set_opacity_mlp", "m1_mlp_train",
           "m1_mlp_get", "m1_mlp_gradient", "m1_opacity_eval", "m1_max_dt", "m1_step_explicit", "m1_step_implicit", "m1_step_rk2",
           "m1_transported", "m1_refresh_opacity", "m1_sync", "m1_diagnostics", "m1_last_error",
           "m1_set_boundary_state", "m1_set_irradiation", "m1_set_groups", "m1_step_noalloc")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library {LIB_PATH} is not built; run python -m paper_2606_26268_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        sig = {
            "m1_params_default": [C.c_double, C.POINTER(m1_params)],
            "m1_create": [C.POINTER(m1_grid), C.c_int, C.c_double, C.POINTER(m1_params), C.POINTER(vp)],
            "m1_destroy": [vp],
            "m1_set_stream": [vp, vp],
            "m1_bind_state": [vp, C.POINTER(m1_fields)],
            "m1_set_opacity_model": [vp, C.c_int, dp],
            "m1_set_opacity_table": [vp, C.c_int, C.c_int] + [C.c_double] * 6 +
                                    [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_double],
            "m1_set_opacity_mlp": [vp, C.POINTER(m1_mlp)],
            "m1_mlp_train": [vp, C.POINTER(m1_train_cfg), C.POINTER(m1_train_report)],
            "m1_mlp_get": [vp, C.POINTER(C.c_float), dp],
            "m1_mlp_gradient": [vp, vp, C.c_long, C.POINTER(C.c_float), C.POINTER(C.c_float), dp],
            "m1_opacity_eval": [vp, C.c_long, vp, vp, vp, vp],
            "m1_max_dt": [vp, C.c_double, dp],
            "m1_step_explicit": [vp, C.c_double],
            "m1_step_implicit": [vp, C.c_double],
            "m1_step_rk2": [vp, C.c_double],
            "m1_step_noalloc": [vp, C.POINTER(m1_fields), C.c_double],
            "m1_transported": [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp)],
            "m1_refresh_opacity": [vp],
            "m1_sync": [vp],
            "m1_diagnostics": [vp, C.POINTER(m1_diag)],
            "m1_set_boundary_state": [vp, C.c_int, C.c_int, dp],
            "m1_set_irradiation": [vp, vp],
            "m1_set_groups": [vp, C.c_int, dp, dp, dp, C.c_double],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.m1_last_error.argtypes = []
        L.m1_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def m1_last_error():
    return lib().m1_last_error().decode()


def _check(status):
    if status != M1_OK:
        raise M1Error(status, m1_last_error())
    return status


# ---------------------------------------------------------------------------
# one wrapper per C call
# ---------------------------------------------------------------------------

def m1_params_default(c_hat):
    p = m1_params()
    _check(lib().m1_params_default(float(c_hat), C.byref(p)))
    return p


def m1_create(ndim, n, faces, bc, geometry, c_hat, params=None):
    """faces: three float64 arrays (host, copied by the library); returns ctx."""
    g = m1_grid()
    g.ndim = int(ndim)
    keep = []
    for d in range(3):
        g.n[d] = int(n[d])
        f = np.ascontiguousarray(faces[d], dtype=np.float64)
        keep.append(f)
        g.faces[d] = f.ctypes.data_as(C.POINTER(C.c_double))
        g.bc[d][0], g.bc[d][1] = int(bc[d][0]), int(bc[d][1])
    ctx = C.c_void_p()
    _check(lib().m1_create(C.byref(g), int(geometry), float(c_hat),
                           C.byref(params) if params is not None else None, C.byref(ctx)))
    return ctx


def m1_destroy(ctx):
    _check(lib().m1_destroy(ctx))


def m1_set_stream(ctx, stream_ptr):
    _check(lib().m1_set_stream(ctx, C.c_void_p(int(stream_ptr)) if stream_ptr else None))


def m1_bind_state(ctx, tensors):
    f = m1_fields()
    for k in ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg"):
        setattr(f, k, C.c_void_p(tensors[k].data_ptr()))
    _check(lib().m1_bind_state(ctx, C.byref(f)))


def m1_set_opacity_model(ctx, kind, params):
    p = np.ascontiguousarray(params, dtype=np.float64)
    _check(lib().m1_set_opacity_model(ctx, int(kind), p.ctypes.data_as(C.POINTER(C.c_double))))


def m1_set_opacity_table(ctx, nr, nt, lr0, lr1, lt0, lt1, lr_off, lt_off, log10_kP, log10_kR, sigma):
    a = np.ascontiguousarray(log10_kP, dtype=np.float32)
    b = np.ascontiguousarray(log10_kR, dtype=np.float32)
    assert a.shape == (nt, nr) and b.shape == (nt, nr)
    fp = C.POINTER(C.c_float)
    _check(lib().m1_set_opacity_table(ctx, int(nr), int(nt), lr0, lr1, lt0, lt1, lr_off, lt_off,
                                      a.ctypes.data_as(fp), b.ctypes.data_as(fp), float(sigma)))


def m1_set_opacity_mlp(ctx, theta, norm):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    assert th.size == M1_MLP_NPARAM
    w = m1_mlp()
    w.theta = th.ctypes.data_as(C.POINTER(C.c_float))
    for i in range(4):
        w.norm[i] = float(norm[i])
    _check(lib().m1_set_opacity_mlp(ctx, C.byref(w)))


def m1_mlp_train(ctx, samples_dev, n_train, n_eval, theta_init, batch=512, steps=20000, lr=3e-3,
                 lr_final=1e-5, beta1=0.9, beta2=0.999, eps=1e-8, keep_init=False):
    th = np.ascontiguousarray(theta_init, dtype=np.float32)
    cfg = m1_train_cfg()
    cfg.samples = C.c_void_p(samples_dev.data_ptr())
    cfg.n_train, cfg.n_eval = int(n_train), int(n_eval)
    cfg.theta_init = th.ctypes.data_as(C.POINTER(C.c_float))
    cfg.batch, cfg.steps = int(batch), int(steps)
    cfg.lr, cfg.lr_final, cfg.beta1, cfg.beta2, cfg.eps = lr, lr_final, beta1, beta2, eps
    cfg.keep_init = int(bool(keep_init))
    rep = m1_train_report()
    _check(lib().m1_mlp_train(ctx, C.byref(cfg), C.byref(rep)))
    return dict(final_loss=rep.final_loss, max_rel_err_P=rep.max_rel_err_P,
                max_rel_err_R=rep.max_rel_err_R, seconds=rep.seconds)


def m1_mlp_get(ctx):
    th = np.zeros(M1_MLP_NPARAM, dtype=np.float32)
    norm = np.zeros(4)
    _check(lib().m1_mlp_get(ctx, th.ctypes.data_as(C.POINTER(C.c_float)),
                            norm.ctypes.data_as(C.POINTER(C.c_double))))
    return th, norm


def m1_mlp_gradient(ctx, samples_dev, n, theta):
    th = np.ascontiguousarray(theta, dtype=np.float32)
    g = np.zeros(M1_MLP_NPARAM, dtype=np.float32)
    loss = C.c_double()
    fp = C.POINTER(C.c_float)
    _check(lib().m1_mlp_gradient(ctx, C.c_void_p(samples_dev.data_ptr()), int(n), th.ctypes.data_as(fp),
                                 g.ctypes.data_as(fp), C.byref(loss)))
    return loss.value, g


def m1_opacity_eval(ctx, n, rho, T, kP, kR):
    assert rho.numel() >= n and T.numel() >= n and kP.numel() >= n and kR.numel() >= n
    _check(lib().m1_opacity_eval(ctx, n, C.c_void_p(rho.data_ptr()), C.c_void_p(T.data_ptr()),
                                 C.c_void_p(kP.data_ptr()), C.c_void_p(kR.data_ptr())))


def m1_max_dt(ctx, cfl):
    dt = C.c_double()
    _check(lib().m1_max_dt(ctx, float(cfl), C.byref(dt)))
    return dt.value


def m1_set_groups(ctx, m, edges, kP, kR, sigma=0.0):
    e = np.ascontiguousarray(edges if m > 1 else [0.0], dtype=np.float64)
    a = np.ascontiguousarray(kP, dtype=np.float64)
    b = np.ascontiguousarray(kR, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    _check(lib().m1_set_groups(ctx, int(m), e.ctypes.data_as(dp), a.ctypes.data_as(dp), b.ctypes.data_as(dp),
                               float(sigma)))


def m1_set_boundary_state(ctx, direction, side, state):
    st = (C.c_double * 4)(*[float(v) for v in state])
    _check(lib().m1_set_boundary_state(ctx, int(direction), int(side), st))


def m1_set_irradiation(ctx, q):
    """q: CUDA float64 tensor of the cell count (or None to switch off); the
    caller keeps it alive while it is set."""
    _check(lib().m1_set_irradiation(ctx, None if q is None else q.data_ptr()))


def m1_step_explicit(ctx, dt):
    _check(lib().m1_step_explicit(ctx, float(dt)))


def m1_step_implicit(ctx, dt):
    _check(lib().m1_step_implicit(ctx, float(dt)))


def m1_step_rk2(ctx, dt):
    _check(lib().m1_step_rk2(ctx, float(dt)))


def m1_step_noalloc(ctx, tensors, dt):
    """One step of the state in `tensors` (E, Fx, Fy, Fz, rho, mx, my, mz,
    Eg device tensors, updated in place) with the library's static buffer."""
    f = m1_fields()
    for k in ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg"):
        setattr(f, k, C.c_void_p(tensors[k].data_ptr()))
    _check(lib().m1_step_noalloc(ctx, C.byref(f), float(dt)))


def m1_transported(ctx):
    ptrs = [C.c_void_p() for _ in range(4)]
    _check(lib().m1_transported(ctx, *[C.byref(p) for p in ptrs]))
    return [p.value for p in ptrs]


def m1_refresh_opacity(ctx):
    _check(lib().m1_refresh_opacity(ctx))


def m1_sync(ctx):
    _check(lib().m1_sync(ctx))


def m1_diagnostics(ctx):
    d = m1_diag()
    _check(lib().m1_diagnostics(ctx, C.byref(d)))
    return dict(rad_energy=d.rad_energy, total_energy=d.total_energy, momentum=list(d.momentum),
                min_E=d.min_E, max_f=d.max_f, counters=list(d.counters))


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

RAD = ("E", "Fx", "Fy", "Fz")
GAS = ("rho", "mx", "my", "mz", "Eg")


class Solver:
    """Device state of one problem plus a library context.

    prob: ``inputs.Problem`` (fields as numpy arrays, or device tensors that
    are used in place); precision: "p64" or "f32"; mlp: optional
    dict(theta=float32[4486], norm=4 floats) for the MLP opacity kind;
    second_order: allocate the buffer of the second-order step at binding
    (needed by step(..., rk2=True)).
    """

    def __init__(self, prob, precision="p64", device="cuda:0", mlp=None, stream=None, second_order=False):
        self.prob = prob
        self.device = torch.device(device)
        self.precision = M1_F32 if precision == "f32" else M1_P64
        rdt = torch.float32 if self.precision == M1_F32 else torch.float64
        self.t = {}

        def dev(a, dt):
            # numpy arrays are copied to the device; device tensors are taken
            # as they are (converted only if the dtype differs)
            if isinstance(a, torch.Tensor):
                return a.to(self.device, dt).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a)).to(self.device, dt).contiguous()

        for k in RAD:
            self.t[k] = dev(prob.fields[k], rdt)
        for k in GAS:
            self.t[k] = dev(prob.fields[k], torch.float64)
        par = m1_params_default(prob.c_hat)
        par.c, par.a_rad, par.gamma = prob.c, prob.a_rad, prob.gamma
        par.precision, par.e_floor = self.precision, prob.e_floor
        par.recon, par.riemann = getattr(prob, "recon", 0), getattr(prob, "riemann", 0)
        par.absorb_only = int(getattr(prob, "absorb_only", 0))
        par.second_order = int(bool(second_order))
        par.limiter = int(getattr(prob, "limiter", 0))
        par.stream_reads = int(getattr(prob, "stream_reads", 0))
        self.ctx = m1_create(prob.ndim, prob.n, prob.faces, prob.bc, prob.geometry, prob.c_hat, par)
        bs = getattr(prob, "bc_state", None)
        if bs is not None:
            for d in range(3):
                for side in range(2):
                    if bs[d][side] is not None:
                        m1_set_boundary_state(self.ctx, d, side, bs[d][side])
        irr = getattr(prob, "irr", None)
        self.irr = None
        if irr is not None:
            self.irr = torch.from_numpy(np.ascontiguousarray(irr, dtype=np.float64)).to(self.device).contiguous()
            m1_set_irradiation(self.ctx, self.irr)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        m1_set_stream(self.ctx, self.stream.cuda_stream)
        op = prob.opacity
        kind = op["kind"]
        if kind == 0:
            m1_set_opacity_model(self.ctx, M1_OPAC_CONSTANT, [op["kP"], op["kR"], op.get("sigma", 0.0)])
        elif kind == 1:
            m1_set_opacity_model(self.ctx, M1_OPAC_POWERLAW,
                                 [op["k0"], op["rho0"], op["alpha"], op["T0"], op["beta"], op.get("sigma", 0.0)])
        else:
            m1_set_opacity_table(self.ctx, op["nr"], op["nt"], op["lr0"], op["lr1"], op["lt0"], op["lt1"],
                                 op["lr_off"], op["lt_off"], op["log10_kP"], op["log10_kR"], op.get("sigma", 0.0))
            if kind == 3:
                if mlp is None:
                    raise ValueError("MLP opacity needs weights (or call train_mlp)")
                m1_set_opacity_mlp(self.ctx, mlp["theta"], mlp["norm"])
        grp = getattr(prob, "groups", None)
        if grp is not None and len(grp["kP"]) > 1:
            m1_set_groups(self.ctx, len(grp["kP"]), grp["edges"], grp["kP"], grp["kR"], op.get("sigma", 0.0))
        m1_bind_state(self.ctx, self.t)

    def close(self):
        if self.ctx is not None:
            m1_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, dt, n=1, rk2=False):
        for _ in range(n):
            if rk2:
                m1_step_rk2(self.ctx, dt)
            else:
                m1_step_explicit(self.ctx, dt)
                m1_step_implicit(self.ctx, dt)

    def sync(self):
        m1_sync(self.ctx)

    def state(self):
        self.sync()
        return {k: v.detach().to("cpu", torch.float64).numpy().reshape(self.prob.fields[k].shape)
                for k, v in self.t.items()}

    def transported(self):
        """Host copy of the library's transported state (E*, F*)."""
        self.sync()
        ptrs = m1_transported(self.ctx)
        n = self.prob.ncells
        typestr = "<f4" if self.precision == M1_F32 else "<f8"
        out = {}
        for k, p in zip(RAD, ptrs):
            view = torch.as_tensor(_DeviceArray(p, n, typestr), device=self.device)
            out[k] = view.to("cpu", torch.float64).numpy().reshape(self.prob.shape)
        return out

    def diagnostics(self):
        return m1_diagnostics(self.ctx)

    def max_dt(self, cfl):
        return m1_max_dt(self.ctx, cfl)


class _DeviceArray:
    """Read-only view of library-owned device memory for torch.as_tensor."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3, "strides": None}
