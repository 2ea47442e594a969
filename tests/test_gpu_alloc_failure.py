"""Allocation failures leave the context usable (C ABI, on the GPU).

A real device allocation failure is produced by first holding all free
device memory in torch tensors and handing a known amount back (no kernel
touches the held memory).  Then:

* a rebinding whose scratch allocation fails, and one whose second-order
  buffer allocation fails after the scratch succeeded, return M1_ENOMEM and
  keep the previous binding: the steps that follow still update the first
  set of arrays, bit for bit like an untouched context;
* a table upload whose allocation fails returns M1_ENOMEM and keeps the
  previous table.
"""
import numpy as np
import pytest

from gpu_common import say

pytestmark = pytest.mark.gpu

MB = 1 << 20


def _problem(n=128):
    from paper_2606_26268_amd import inputs as I
    faces = [I.uniform_faces(n, 0.0, 1.0) for _ in range(3)]
    p = I.make_random_state(I.CARTESIAN, (n, n, n), 3, 11, faces, [[I.PERIODIC] * 2] * 3,
                            fmax=0.8, c_hat=2.0)
    p.dt = 0.4 / (2.0 * 3 * n)
    return p


def _fields(m1, t):
    f = m1.m1_fields()
    for k in ("E", "Fx", "Fy", "Fz", "rho", "mx", "my", "mz", "Eg"):
        setattr(f, k, m1.C.c_void_p(t[k].data_ptr()))
    return f


def _fp(m1, a):
    return a.ctypes.data_as(m1.C.POINTER(m1.C.c_float))


class DeviceFill:
    """Holds all free device memory in torch tensors (1 GiB chunks, then
    16 MiB chunks until an allocation fails), then hands `keep` MiB back in
    16 MiB chunks: afterwards between keep and keep + 16 MiB are free.  Each
    chunk is its own device allocation (above torch's small-block sizes),
    so releasing it and emptying torch's cache returns it to the device.
    Everything is released on exit, whatever happened inside."""

    def __init__(self, torch, keep_mib):
        self.torch, self.keep = torch, keep_mib
        self.chunks = []

    def __enter__(self):
        torch = self.torch
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for size in (1024 * MB, 16 * MB):
            while True:
                try:
                    self.chunks.append(torch.empty(size, dtype=torch.uint8, device="cuda"))
                except RuntimeError:          # torch.OutOfMemoryError and HIP errors
                    break
        small = [c for c in self.chunks if c.numel() == 16 * MB]
        give = self.keep // 16
        assert len(small) >= give, "could not fill the device in 16 MiB chunks"
        drop = {id(c) for c in small[:give]}
        self.chunks = [c for c in self.chunks if id(c) not in drop]
        del small
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return self

    def __exit__(self, *exc):
        self.chunks.clear()
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()
        return False


def test_failed_rebind_keeps_the_previous_binding():
    import torch
    from paper_2606_26268_amd import m1
    p = _problem()
    ref = m1.Solver(p, "p64", second_order=True)
    s = m1.Solver(p, "p64", second_order=True)
    # scratch: 6 fields of 16.8 MB (~101 MB); second-order buffer ~134 MB
    spare = {k: v.clone() for k, v in s.t.items()}
    torch.cuda.synchronize()
    # with 64-80 MiB free the scratch fails; with 160-176 MiB free the
    # scratch fits and the second-order buffer after it does not
    for keep, what in ((64, "scratch"), (160, "second-order buffer")):
        say(f"  rebinding with {keep}-{keep + 16} MiB free: the {what} allocation fails")
        with DeviceFill(torch, keep):
            status = m1.lib().m1_bind_state(s.ctx, m1.C.byref(_fields(m1, spare)))
            msg = m1.m1_last_error()
        assert status == m1.M1_ENOMEM, (status, msg)
        assert what in msg, msg
    before = {k: v.clone() for k, v in spare.items()}
    for solver in (ref, s):
        solver.step(p.dt, 2)
        solver.step(p.dt, 2, rk2=True)
    a, b = ref.state(), s.state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    for k in spare:
        assert torch.equal(spare[k], before[k]), k
    assert s.diagnostics()["counters"] == ref.diagnostics()["counters"]
    ref.close()
    s.close()


def test_failed_table_upload_keeps_the_previous_table():
    import torch
    from paper_2606_26268_amd import inputs as I
    from paper_2606_26268_amd import m1
    q = I.make_c3(nr=24, nth=12, nph=16, dt=2e-5)
    ref = m1.Solver(q, "f32")
    s = m1.Solver(q, "f32")
    # a 4096 x 4096 table (2 x 64 MiB) cannot be allocated in 64-80 MiB
    big = np.zeros((4096, 4096), dtype=np.float32)
    op = q.opacity
    with DeviceFill(torch, 64):
        status = m1.lib().m1_set_opacity_table(s.ctx, 4096, 4096, op["lr0"], op["lr1"], op["lt0"], op["lt1"],
                                               op["lr_off"], op["lt_off"], _fp(m1, big), _fp(m1, big), 0.0)
        msg = m1.m1_last_error()
    assert status == m1.M1_ENOMEM, (status, msg)
    for solver in (ref, s):
        solver.step(q.dt, 3)
    a, b = ref.state(), s.state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    ref.close()
    s.close()
