"""Write tests/golden/shock_tube_reference_<tube>.npz: the radiation energy
and flux of the optically thin shock tubes of Sect. 3.1 at t = 20, from the
oracle with N_REF cells, second-order (RK2) steps at Courant number 0.4 and
the PLM reconstruction with the f-preserving face fix (the paper's reference
solutions are PLM runs at 2^17 cells), stored as averages over N_OUT coarse
cells.  It calls only the oracle and the shared input generator.

    python tests/golden/make_shock_tube_reference.py [N_REF [TUBE ...]]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2606_26268_amd import inputs as I  # noqa: E402

N_OUT = 4096


def main():
    n_ref = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 15
    tubes = [int(a) for a in sys.argv[2:]] or [1, 2]
    for which in tubes:
        p = I.make_shock_tube(which, N=n_ref)
        t0 = time.perf_counter()
        st, cnt = orc.Oracle(p).run(p.fields, p.dt, p.steps, rk2=True)
        assert st["E"].min() > 0 and (cnt[:3] == 0).all(), cnt
        out = {"n_ref": n_ref, "n_out": N_OUT, "t_end": 20.0, "cfl": 0.4, "steps": p.steps}
        for k in ("E", "Fx", "Fy"):
            out[k] = st[k][0, 0].reshape(N_OUT, n_ref // N_OUT).mean(axis=1)
        np.savez_compressed(os.path.join(HERE, f"shock_tube_reference_{which}.npz"), **out)
        print(f"tube {which}: {n_ref} cells, {p.steps} RK2 steps, {time.perf_counter() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
